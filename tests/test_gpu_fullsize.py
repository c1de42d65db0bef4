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
# stored level-3 samples (tests/golden/make_golden.py c2, span): the first two, the extreme
# recharge zeta (68 min, 313 max), the largest and smallest log-permeability contrast (342, 502),
# the largest porosity contrast (478) and the last index of the batch (511)
C2_SAMPLES = (0, 1, 68, 313, 342, 478, 502, 511)


def _run(name, prec, **okw):
    import paper_2403_17018_amd as P
    w = WORKLOADS[name]
    th = draw_theta(w["seed"], w["nsamples"], level=w["level"])
    hx = P.Henry(0)
    g = P.grid(*level_grid(w["level"]))
    r = hx.solve(torch.from_numpy(th).cuda(), g, opts=P.solver_opts(mg_precision=prec, **okw), want_c=True,
                 want_p=True)
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
    from oracle import henry as H
    ny, nx = out["c"].shape[:2]
    bf, bs = defect_bound(out["theta"], H.Problem(), nx, ny, out["nsteps"])
    assert (out["st"][:, 2] < bf).all() and (out["st"][:, 3] < bs).all()
    assert out["c"].min() >= -1e-10 and out["c"].max() <= 1 + 1e-10


def test_level3_fp64_full_batch():
    """256x128 cells, 384 steps, all 512 samples of seed 1 in one batch (the benchmark workload)."""
    _check(_run("c2_fp64_level3", 64), "c2", C2_SAMPLES)


def test_level3_named_configuration_32x16_dense_lu():
    """The workload as named: multigrid down to a 32x16 coarsest grid (4 grids from 256x128)
    solved by the batched dense LU with partial pivoting, all 512 samples in one batch."""
    _check(_run("c2_fp64_level3", 64, coarse_nx=32, coarse_ny=16, coarse_solver=1), "c2", C2_SAMPLES)


def test_level3_named_configuration_32x16_pivoted_band_lu():
    """The same 32x16 coarsest grid solved by Gaussian elimination with partial pivoting in band
    storage (the dense elimination's pivots and factors, without its O(n^3) work)."""
    _check(_run("c2_fp64_level3", 64, coarse_nx=32, coarse_ny=16, coarse_solver=2), "c2", C2_SAMPLES)


def test_level3_fp32_multigrid_full_batch():
    """Same workload with the FP32 multigrid preconditioner inside FP64 BiCGStab/Newton."""
    _check(_run("c2_fp64_level3", 32), "c2", C2_SAMPLES)


def test_level4_fp32_multigrid_full_batch():
    """512x256 cells, 768 steps, 128 samples of seed 2 with the FP32 multigrid preconditioner, against
    the stored oracle runs of samples 0, 84 (smallest zeta) and 127 (the last)."""
    _check(_run("c3_mixed_level4", 32), "c3", (0, 84, 127))


def test_mlmc_hierarchy_full_run():
    """Levels 0..4 with 4096/1024/256/64/16 samples and their coupled coarse partners
    (seed 3), in one ragged call with hipGraphs, as the benchmark times it.  Sampled
    realisations of every grid against the oracle (levels 0 and 1 run live, levels 2 and 3
    stored), every sample against the invariants, and the estimate against the oracle's
    estimator (eq. A, the variance sum, the bias bound and the fields) on the same QoIs."""
    import paper_2403_17018_amd as P
    from oracle import mlmc as M
    from tests.oracle_runs import oracle_batch
    w = WORKLOADS["c4_mlmc_levels0to4"]
    levels, m, seed = w["levels"], w["nsamples"], w["seed"]
    ths = [draw_theta(seed, k, level=l) for l, k in zip(levels, m)]
    hx = P.Henry(0)
    est = P.mlmc_run(hx, [torch.from_numpy(t).cuda() for t in ths], levels, opts=P.solver_opts(use_graphs=1))
    torch.cuda.synchronize()
    assert est["nfailed"] == 0
    res = est["results"]   # level 0 fine; then per level l >= 1: fine, coarse partner
    fine = [res[0]] + [res[2 * l - 1] for l in range(1, len(levels))]
    coarse = [None] + [res[2 * l] for l in range(1, len(levels))]
    host = lambda r: dict(c=r.c_T.permute(2, 0, 1).cpu().numpy(), q=r.qoi.cpu().numpy(), st=r.stats.cpu().numpy())
    F = [host(r) for r in fine]
    Cp = [None] + [host(r) for r in coarse[1:]]
    hx.close()

    def same(c, q, ref_c, ref_q, what):
        assert np.abs(c.ravel() - ref_c.ravel()).max() <= TOL * np.abs(ref_c).max(), what
        assert abs(q - ref_q) <= TOL * abs(ref_q), what

    # live oracle: level-0 samples 0 and 4095, level-1 samples 0 and 1023 and the coarse
    # partner of level-1 sample 0 (its theta on the level-0 grid)
    r0 = oracle_batch(np.stack([ths[0][0], ths[0][-1], ths[1][0]]), 32, 16, 48)
    r1 = oracle_batch(np.stack([ths[1][0], ths[1][-1]]), 64, 32, 96)
    same(F[0]["c"][0], F[0]["q"][0], r0["c"][0], r0["qoi"][0], "level 0, sample 0")
    same(F[0]["c"][-1], F[0]["q"][-1], r0["c"][1], r0["qoi"][1], "level 0, last sample")
    same(Cp[1]["c"][0], Cp[1]["q"][0], r0["c"][2], r0["qoi"][2], "level 1 coarse partner, sample 0")
    same(F[1]["c"][0], F[1]["q"][0], r1["c"][0], r1["qoi"][0], "level 1, sample 0")
    same(F[1]["c"][-1], F[1]["q"][-1], r1["c"][1], r1["qoi"][1], "level 1, last sample")
    # stored oracle results (tests/golden/make_golden.py c4)
    for name, arr in (("c4_l2", F[2]), ("c4_l3", F[3]), ("c4_l4coarse", Cp[4])):
        z = np.load(os.path.join(GOLD, f"oracle_{name}_s0.npz"))
        src = ths[4][0] if name == "c4_l4coarse" else ths[int(name[-1])][0]
        assert np.array_equal(z["theta"], src)
        same(arr["c"][0], arr["q"][0], z["c_T"], float(z["qoi"]), name)
    # invariants of every sample of every grid
    for l, lev in enumerate(levels):
        for out, glev in ((F[l], lev), (Cp[l], lev - 1)):
            if out is None:
                continue
            from oracle import henry as H
            bf, bs = defect_bound(ths[l], H.Problem(), 32 << glev, 16 << glev, 48 << glev)
            assert (out["st"][:, 2] < bf).all() and (out["st"][:, 3] < bs).all(), (l, glev)
            assert out["c"].min() >= -1e-10 and out["c"].max() <= 1 + 1e-10, (l, glev)
    # the estimator on the same QoIs and fields
    ref = M.estimate([f["q"] for f in F], [None if c is None else c["q"] for c in Cp])
    assert est["mean"] == pytest.approx(ref["mean"], rel=1e-12)
    assert np.allclose(est["V"], ref["V"], rtol=1e-9, atol=0.0)
    assert est["rmse"] == pytest.approx(ref["rmse"], rel=1e-9)
    mf, vf = M.field_estimate([f["c"] for f in F], [None if c is None else c["c"] for c in Cp])
    assert np.abs(est["mean_field"].cpu().numpy() - mf).max() <= 1e-11
    assert np.abs(est["var_field"].cpu().numpy() - vf).max() <= 1e-11


def test_vc_level1_paper_full_batch():
    """The paper's vertex-centred discretisation on level 1 of Table 2 (64 x 32 elements, 2145
    vertices, 376 steps) with its section-4 model: all 512 samples of seed 5 in one batch (the
    benchmark's configuration), against the stored vertex-oracle runs of samples 0, the smallest
    and largest recharge zeta of the first 128 (7, 63) and of all 512 (300, 389), and the last
    indices 127 and 511; every sample converged with c in [0, 1]."""
    import paper_2403_17018_amd as P
    th = draw_theta(5, 512)
    hx = P.Henry(0)
    g = P.vc_level_grid(1)
    r = hx.vc_solve(torch.from_numpy(th).cuda(), g, P.paper_problem(),
                    P.solver_opts(krylov_maxit=1000, nu_pre=1, nu_post=1, use_graphs=1),
                    want_c=True, want_p=True)
    torch.cuda.synchronize()
    c, p, q = r.c_T.cpu().numpy(), r.p_T.cpu().numpy(), r.qoi.cpu().numpy()
    hx.close()
    assert r.nfailed == 0
    for s in (0, 7, 63, 127, 300, 389, 511):
        z = np.load(os.path.join(GOLD, f"oracle_f3_l1_s{s}.npz"))
        assert np.array_equal(z["theta"], th[s]) and bool(z["converged"])
        assert np.abs(c[..., s].ravel() - z["c_T"]).max() <= TOL * np.abs(z["c_T"]).max(), s
        assert np.abs(p[..., s].ravel() - z["p_T"]).max() <= TOL * np.abs(z["p_T"]).max(), s
        assert abs(q[s] - float(z["qoi"])) <= TOL * abs(float(z["qoi"])), s
    assert c.min() >= -1e-9 and c.max() <= 1 + 1e-9
