"""GPU parity for the paper's own stochastic model (section 4): two-layer multiscale
porosity (eq. poro_2levels), Kozeny-Carman permeability (eq. e_perm_Kozeny_Carman) and the
periodic recharge (eq. e_recharge_of_param), T = 6016 s.  Same tolerance as the KL model:
per sample max|c_gpu - c_oracle| / max|c_oracle| <= 1e-8, likewise p and the QoI."""
import math
import os

import numpy as np
import pytest
import torch

from henry_inputs import draw_theta, level_grid
from tests.oracle_runs import defect_bound, oracle_batch, rel_inf

pytestmark = pytest.mark.gpu
TOL = 1e-8
GOLD = os.path.join(os.path.dirname(__file__), "golden")
ORACLE_KW = dict(field_model="paper", q_in_amp=0.5, recharge_omega=math.pi / 40.0, T=6016.0)


@pytest.fixture(scope="module")
def hx():
    import paper_2403_17018_amd as P
    h = P.Henry(0)
    yield h
    h.close()


def _oracle_prob():
    from oracle import henry as H
    return H.paper_problem()


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _solve(hx, th, g, **okw):
    import paper_2403_17018_amd as P
    r = hx.solve(_cuda(th), g, P.paper_problem(), P.solver_opts(**okw), want_c=True, want_p=True)
    torch.cuda.synchronize()
    return r, r.c_T.permute(2, 0, 1).cpu().numpy(), r.p_T.permute(2, 0, 1).cpu().numpy()


def test_paper_fields_match_oracle(hx):
    """Level 2 (the small scales sin(64 pi x), sin(32 pi y) resolved) and level 4."""
    import paper_2403_17018_amd as P
    from oracle import henry as H
    th = draw_theta(5, 19)
    for lev in (2, 4):
        g = P.level_grid(lev)
        phi, K, q = hx.sample_fields(_cuda(th), g, P.paper_problem())
        phi, K, q = (t.cpu().numpy() for t in (phi, K, q))
        for s in (0, 7, 18):
            rphi, rK, ru = H.sample_fields(H.paper_problem(), H.Grid(g.nx, g.ny, g.nsteps), th[s])
            assert np.abs(phi[..., s] - rphi).max() <= 1e-14
            assert np.abs(K[..., s] / rK - 1).max() <= 1e-12
            assert abs(q[s] - ru) <= 1e-18


@pytest.mark.parametrize("level", [0, 1])
def test_paper_model_matches_oracle(hx, level):
    """Levels 0 and 1 over the paper's horizon (48 and 96 steps of 6016 s), 8 samples."""
    import paper_2403_17018_amd as P
    th = draw_theta(5, 8, level=level)
    g = P.level_grid(level)
    # FP64 and FP32 multigrid with the default first guess (the inflow-aware one), and the
    # plain linear extrapolation: the guess changes the iteration path, not the fixed point
    for prec, ext in ((64, 2), (32, 2), (64, 1)):
        r, c, p = _solve(hx, th, g, mg_precision=prec, newton_extrapolate=ext)
        ref = oracle_batch(th, g.nx, g.ny, g.nsteps, ORACLE_KW)
        assert r.nfailed == 0 and ref["conv"].all()
        assert rel_inf(c, ref["c"]).max() <= TOL, (prec, ext)
        assert rel_inf(p, ref["p"]).max() <= TOL, (prec, ext)
        q = r.qoi.cpu().numpy()
        assert np.abs(q - ref["qoi"]).max() <= TOL * np.abs(ref["qoi"]).max()
        st = r.stats.cpu().numpy()
        bf, bs = defect_bound(th, _oracle_prob(), g.nx, g.ny, g.nsteps)
        assert (st[:, 2] < bf).all() and (st[:, 3] < bs).all()
        assert c.min() >= -1e-10 and c.max() <= 1 + 1e-10


def test_paper_model_level2_batch_against_stored_oracle(hx):
    """Level 2 (128x64 cells, 192 steps), 64 samples of seed 5 in one batch: samples 0 and 1
    against the stored oracle results (tests/golden/make_golden.py f1), invariants for all."""
    import paper_2403_17018_amd as P
    th = draw_theta(5, 64, level=2)
    r, c, p = _solve(hx, th, P.level_grid(2))
    assert r.nfailed == 0
    q = r.qoi.cpu().numpy()
    for s in (0, 1):
        z = np.load(os.path.join(GOLD, f"oracle_f1_s{s}.npz"))
        assert np.array_equal(z["theta"], th[s])
        assert np.abs(c[s].ravel() - z["c_T"]).max() <= TOL * np.abs(z["c_T"]).max()
        assert np.abs(p[s].ravel() - z["p_T"]).max() <= TOL * np.abs(z["p_T"]).max()
        assert abs(q[s] - float(z["qoi"])) <= TOL * abs(float(z["qoi"]))
    st = r.stats.cpu().numpy()
    bf, bs = defect_bound(th, _oracle_prob(), 128, 64, 192)
    assert (st[:, 2] < bf).all() and (st[:, 3] < bs).all()
    assert c.min() >= -1e-10 and c.max() <= 1 + 1e-10


def test_paper_model_benchmark_batch_against_stored_oracle(hx):
    """The benchmark's paper-model line in its launch configuration: 256x128 cells, 384 steps
    over T = 6016 s, all 512 samples of seed 1 in one batch.  Sample 0 against the stored
    oracle result (tests/golden/make_golden.py f1l3), invariants for every sample."""
    import paper_2403_17018_amd as P
    th = draw_theta(1, 512, level=3)
    r, c, p = _solve(hx, th, P.level_grid(3))
    assert r.nfailed == 0
    z = np.load(os.path.join(GOLD, "oracle_f1l3_s0.npz"))
    assert np.array_equal(z["theta"], th[0])
    assert np.abs(c[0].ravel() - z["c_T"]).max() <= TOL * np.abs(z["c_T"]).max()
    assert np.abs(p[0].ravel() - z["p_T"]).max() <= TOL * np.abs(z["p_T"]).max()
    assert abs(float(r.qoi[0]) - float(z["qoi"])) <= TOL * abs(float(z["qoi"]))
    st = r.stats.cpu().numpy()
    bf, bs = defect_bound(th, _oracle_prob(), 256, 128, 384)
    assert (st[:, 2] < bf).all() and (st[:, 3] < bs).all()
    assert c.min() >= -1e-10 and c.max() <= 1 + 1e-10


def test_recharge_pressure_closed_form(hx):
    """Constant density, uniform phi and K (theta = 0) and the periodic recharge: after the
    last step p = -rho0 g y + mu u_in(T) (Lx - x) / K exactly, u_in(T) = 6.6e-5 (1 + 0.5 zeta)
    (1 + sin(pi T / 40)), the recharge taken at the end of the step."""
    import paper_2403_17018_amd as P
    th = np.zeros((3, 13))
    th[:, 12] = (0.4, -0.3, 0.9)
    g = P.grid(32, 16, 13)
    pr = P.problem(rho1=1000.0, q_in_amp=0.5, recharge_omega=math.pi / 40.0, T=130.0)
    r = hx.solve(_cuda(th), g, pr, P.solver_opts(), want_c=True, want_p=True)
    torch.cuda.synchronize()
    assert r.nfailed == 0
    p = r.p_T.cpu().numpy()
    h = 1.0 / 16
    x = (np.arange(32) + 0.5) * h
    y = -1.0 + (np.arange(16) + 0.5) * h
    for s in range(3):
        u = 6.6e-5 * (1.0 + 0.5 * th[s, 12]) * (1.0 + math.sin(math.pi * 130.0 / 40.0))
        exact = -1000.0 * 9.81 * y[:, None] + 1e-3 * u * (2.0 - x[None, :]) / 1.020408e-9
        assert np.abs(p[..., s] - exact).max() <= 1e-9 * 1000.0 * 9.81
    # no salt enters (outflow everywhere at the right side); inexact Newton iterates may
    # touch c by less than the Newton tolerance
    assert np.abs(r.c_T.cpu().numpy()).max() <= 1e-9


def _oracle_adjoint_paper(th, nx, ny, nsteps, T):
    """Oracle adjoint of the paper's model in a child interpreter (the test process has the GPU open)."""
    import json
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = f"""
import sys, json, numpy as np
sys.path.insert(0, {root!r})
from oracle import henry as H, adjoint as A
th = np.array(json.loads(sys.argv[1]))
pr = H.paper_problem(T={T}); g = H.Grid({nx}, {ny}, {nsteps})
out = [A.adjoint_gradient(pr, g, t) for t in th]
print(json.dumps([[q, list(gr)] for q, gr in out]))
"""
    r = subprocess.run([sys.executable, "-c", code, json.dumps(th.tolist())], capture_output=True, text=True,
                       check=True)
    out = json.loads(r.stdout)
    return np.array([o[0] for o in out]), np.array([o[1] for o in out])


@pytest.mark.parametrize("prec", [64, 32])
def test_adjoint_of_paper_model_matches_oracle_and_fd(hx, prec):
    """dQ/dxi_1, dQ/dxi_2 (porosity and Kozeny-Carman permeability) and dQ/dxi_3 (the
    periodic recharge, a different factor every step) on 32x16 cells, 12 steps over
    T = 1504 s, checkpoints every 5 steps: against the oracle's adjoint and against
    central differences (h = 1e-6) of batched GPU forward solves; the slots the model
    does not use are exactly 0."""
    import paper_2403_17018_amd as P
    th = draw_theta(24, 5, level=1)
    T = 6016.0 * 12 / 48
    prob = P.paper_problem(T=T)
    g = P.grid(32, 16, 12)
    tight = dict(newton_tol=1e-13, krylov_rtol=1e-12, krylov_maxit=200, newton_maxit=60, mg_precision=prec)
    q, gr, st, nf = hx.adjoint(_cuda(th), g, prob, P.solver_opts(**tight), checkpoint_every=5)
    assert nf == 0
    q, gr = q.cpu().numpy(), gr.cpu().numpy()
    qo, go = _oracle_adjoint_paper(th, 32, 16, 12, T)
    assert np.abs(q - qo).max() <= 1e-10 * np.abs(qo).max()
    assert np.all(gr[:, 2:12] == 0.0)
    for s in range(th.shape[0]):
        assert np.abs(gr[s] - go[s]).max() <= 1e-7 * np.abs(go[s]).max(), (s, gr[s], go[s])
    # central differences in the three parameters the model uses, one batched solve
    h = 1e-6
    comps = (0, 1, 12)
    pert = np.repeat(th[:, None, None, :], 2, axis=1).repeat(len(comps), axis=2)
    for a, k in enumerate(comps):
        pert[:, 0, a, k] += h
        pert[:, 1, a, k] -= h
    r = hx.solve(_cuda(pert.reshape(-1, 13)), g, prob, P.solver_opts(**tight), want_c=False)
    assert r.nfailed == 0
    qq = r.qoi.cpu().numpy().reshape(th.shape[0], 2, len(comps))
    fd = (qq[:, 0] - qq[:, 1]) / (2 * h)
    for s in range(th.shape[0]):
        assert np.abs(gr[s][list(comps)] - fd[s]).max() <= 1e-6 * np.abs(fd[s]).max(), (s, gr[s], fd[s])


def test_qmc_estimate_matches_oracle(hx):
    """Quasi-Monte Carlo over Halton points (section 5 uses 600) for the paper's model: one
    level of the estimator gives the mean and variance of the QoI and of the c field at T.
    64 points at level 0 against the oracle's solves and estimator."""
    import paper_2403_17018_amd as P
    from henry_inputs import qmc_theta
    from oracle import mlmc as M
    th = qmc_theta(64)
    est = P.mlmc_run(hx, [_cuda(th)], [0], prob=P.paper_problem())
    assert est["nfailed"] == 0
    ref = oracle_batch(th, 32, 16, 48, ORACLE_KW)
    r = M.estimate([ref["qoi"]], [None])
    assert est["mean"] == pytest.approx(r["mean"], rel=TOL)
    assert est["V"][0] == pytest.approx(r["V"][0], rel=1e-6)
    mf, vf = M.field_estimate([ref["c"]], [None])
    assert np.abs(est["mean_field"].cpu().numpy() - mf).max() <= TOL
    assert np.abs(est["var_field"].cpu().numpy() - vf).max() <= TOL
