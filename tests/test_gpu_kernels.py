"""Kernel-level GPU parity: each kernel of the solve against the oracle or a library routine,
through the kernel-level C ABI calls (one launch of the solve's own kernel each).

  assembly        R and J entrywise against the oracle's residual and analytic Jacobian
  operator        J x and J^T x against the oracle's sparse matrix; <J x, y> = <x, J^T y>
  smoother pass   one red or black 2x2-block Gauss-Seidel pass against a plain CPU pass
  coarse solvers  banded LU and dense pivoted LU (FP64, FP32; plain and transposed) against
                  numpy.linalg.solve, including a matrix that needs row interchanges
and the solve with the 32x16 coarse grid and the dense pivoted LU against the oracle."""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import torch

from henry_inputs import draw_theta
from tests.oracle_runs import oracle_batch, rel_inf

pytestmark = pytest.mark.gpu
PAPER_KW = dict(field_model="paper", q_in_amp=0.5, recharge_omega=math.pi / 40.0, T=6016.0)


@pytest.fixture(scope="module")
def hx():
    import paper_2403_17018_amd as P
    h = P.Henry(0)
    yield h
    h.close()


def _cu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _np(t):
    return t.cpu().numpy()


def _sample_major(a):
    """[..., ny, nx, S] -> [S, ..., ny, nx]"""
    return np.moveaxis(a, -1, 0)


def _states(prob_kw, nx, ny, nsteps, th, rng):
    """Oracle states after steps 2 and 3 of each sample, with noise on p and c (so that faces
    carry flow in both directions): (p, c, c_old) [S, ny, nx] and the oracle's Problem."""
    from oracle import henry as H
    pr = H.Problem(**{k: (bool(v) if k == "right_c_dirichlet" else v) for k, v in prob_kw.items()})
    if prob_kw.get("field_model") == "paper":
        pr = H.paper_problem()
    g = H.Grid(nx, ny, nsteps)
    P, Cc, Co = [], [], []
    for t in th:
        r = H.solve_sample(pr, g, t, nsteps=3, keep_states=True)
        p, c = r.states[3]
        P.append(p.reshape(ny, nx) + 50.0 * rng.normal(size=(ny, nx)))
        Cc.append(np.clip(c.reshape(ny, nx) + 0.2 * rng.uniform(size=(ny, nx)), 0.0, 1.0))
        Co.append(r.states[2][1].reshape(ny, nx))
    return pr, g, np.array(P), np.array(Cc), np.array(Co)


def _blocks_to_sparse(Js, nx, ny):
    """GPU block layout [20][ny][nx] of one sample -> scipy CSR in the oracle's unknown order
    (2 * cell + component)."""
    rows, cols, vals = [], [], []
    for j in range(ny):
        for i in range(nx):
            P = j * nx + i
            for blk, (di, dj) in enumerate(((0, 0), (-1, 0), (1, 0), (0, -1), (0, 1))):
                qi, qj = i + di, j + dj
                if not (0 <= qi < nx and 0 <= qj < ny):
                    assert np.all(Js[blk * 4:blk * 4 + 4, j, i] == 0.0)
                    continue
                Q = qj * nx + qi
                for a in range(2):
                    for b in range(2):
                        rows.append(2 * P + a)
                        cols.append(2 * Q + b)
                        vals.append(Js[blk * 4 + a * 2 + b, j, i])
    n = 2 * nx * ny
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


@pytest.mark.parametrize("model", ["kl", "paper", "dirichlet"])
def test_assembly_matches_oracle_entrywise(hx, model):
    import paper_2403_17018_amd as P
    nx, ny, nsteps, S = 48, 24, 12, 5
    kw = dict(PAPER_KW) if model == "paper" else (dict(right_c_dirichlet=1) if model == "dirichlet" else {})
    rng = np.random.default_rng(17)
    th = draw_theta(71, S, level=1)
    pr, g, p, c, co = _states(kw, nx, ny, nsteps, th, rng)
    step = 5
    gprob = P.paper_problem() if model == "paper" else P.problem(**kw)
    R, J = hx.assemble(_cu(th), P.grid(nx, ny, nsteps), _cu(np.moveaxis(p, 0, -1)), _cu(np.moveaxis(c, 0, -1)),
                       _cu(np.moveaxis(co, 0, -1)), step, gprob)
    R, J = _sample_major(_np(R)), _sample_major(_np(J))
    from oracle import henry as H
    for s in range(S):
        phi, K, u = H.sample_fields(pr, g, th[s])
        d = H.Discretisation(pr, g, phi, K, u)
        d.set_time((step + 1) * d.tau)
        Rp, Rc = d.residual(p[s].ravel(), c[s].ravel(), co[s].ravel())
        for got, want in ((R[s, 0].ravel(), Rp), (R[s, 1].ravel(), Rc)):
            assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max(), (model, s)
        Jo = d.jacobian(p[s].ravel(), c[s].ravel()).toarray()
        Jg = _blocks_to_sparse(J[s], nx, ny).toarray()
        rowmax = np.abs(Jo).max(axis=1, keepdims=True)
        assert (np.abs(Jg - Jo) <= 1e-13 * rowmax).all(), (model, s)


def test_operator_and_transpose_against_oracle(hx):
    import paper_2403_17018_amd as P
    nx, ny, nsteps, S = 40, 20, 10, 7
    rng = np.random.default_rng(18)
    th = draw_theta(72, S, level=1)
    pr, g, p, c, co = _states({}, nx, ny, nsteps, th, rng)
    gg = P.grid(nx, ny, nsteps)
    _, J = hx.assemble(_cu(th), gg, _cu(np.moveaxis(p, 0, -1)), _cu(np.moveaxis(c, 0, -1)),
                       _cu(np.moveaxis(co, 0, -1)), 0)
    x = rng.normal(size=(2, ny, nx, S))
    y = rng.normal(size=(2, ny, nx, S))
    Jx = _np(hx.jacobian_apply(J, _cu(x), gg))
    Jty = _np(hx.jacobian_apply(J, _cu(y), gg, transpose=True))
    Jh = _sample_major(_np(J))
    for s in range(S):
        A = _blocks_to_sparse(Jh[s], nx, ny)
        xs = np.stack([x[0, ..., s].ravel(), x[1, ..., s].ravel()], axis=1).ravel()   # 2 * cell + comp
        ys = np.stack([y[0, ..., s].ravel(), y[1, ..., s].ravel()], axis=1).ravel()
        ax, aty = A @ xs, A.T @ ys
        scale_x = abs(A) @ np.abs(xs)
        scale_y = abs(A).T @ np.abs(ys)
        gx = np.stack([Jx[0, ..., s].ravel(), Jx[1, ..., s].ravel()], axis=1).ravel()
        gy = np.stack([Jty[0, ..., s].ravel(), Jty[1, ..., s].ravel()], axis=1).ravel()
        assert (np.abs(gx - ax) <= 1e-14 * scale_x + 1e-300).all(), s
        assert (np.abs(gy - aty) <= 1e-14 * scale_y + 1e-300).all(), s
        lhs, rhs = gx @ ys, xs @ gy
        assert abs(lhs - rhs) <= 1e-13 * (np.abs(ys) @ scale_x), s


@pytest.mark.parametrize("transpose", [False, True])
def test_gauss_seidel_pass_matches_cpu_pass(hx, transpose):
    import paper_2403_17018_amd as P
    nx, ny, nsteps, S = 33, 18, 10, 6     # odd nx: rows of unequal colour counts
    rng = np.random.default_rng(19)
    th = draw_theta(73, S, level=1)
    gg = P.grid(nx, ny, nsteps)
    prob = P.problem(Lx=nx / 16.0, Ly=ny / 16.0)     # square cells of 1/16 m
    from oracle import henry as H
    pro = H.Problem(Lx=nx / 16.0, Ly=ny / 16.0)
    gro = H.Grid(nx, ny, nsteps)
    Ps, Cs, Cos = [], [], []
    for t in th:
        r = H.solve_sample(pro, gro, t, nsteps=2, keep_states=True)
        Ps.append(r.states[2][0].reshape(ny, nx) + 30.0 * rng.normal(size=(ny, nx)))
        Cs.append(np.clip(r.states[2][1].reshape(ny, nx) + 0.2 * rng.uniform(size=(ny, nx)), 0, 1))
        Cos.append(r.states[1][1].reshape(ny, nx))
    _, J = hx.assemble(_cu(th), gg, _cu(np.moveaxis(np.array(Ps), 0, -1)), _cu(np.moveaxis(np.array(Cs), 0, -1)),
                       _cu(np.moveaxis(np.array(Cos), 0, -1)), 0, prob)
    b = rng.normal(size=(2, ny, nx, S))
    x0 = rng.normal(size=(2, ny, nx, S))
    Jh = _sample_major(_np(J))
    for colour in (0, 1):
        x = _cu(x0)
        hx.gs_pass(J, _cu(b), x, gg, colour, transpose)
        got = _np(x)
        for s in range(S):
            A = _blocks_to_sparse(Jh[s], nx, ny)
            A = (A.T if transpose else A).tocsr()
            xs = np.stack([x0[0, ..., s].ravel(), x0[1, ..., s].ravel()], axis=1).ravel()
            bs = np.stack([b[0, ..., s].ravel(), b[1, ..., s].ravel()], axis=1).ravel()
            want = xs.copy()
            for j in range(ny):
                for i in range(nx):
                    if (i + j) % 2 != colour:
                        continue
                    q = j * nx + i
                    r = slice(2 * q, 2 * q + 2)
                    row = A[r].toarray()
                    D = row[:, r]
                    off = row @ xs - D @ xs[r]          # neighbours keep their old values (other colour)
                    want[r] = np.linalg.solve(D, bs[r] - off)
            gs = np.stack([got[0, ..., s].ravel(), got[1, ..., s].ravel()], axis=1).ravel()
            assert np.abs(gs - want).max() <= 1e-12 * np.abs(want).max(), (colour, s)


def _coarse_case(rng, nx, ny, S, kind):
    """Block operators [20][ny][nx][S] and right-hand sides [2][ny][nx][S]: the oracle's Jacobian
    of a state on that grid ("jacobian"), or random blocks whose first cell has the centre block
    [[0, 1], [1, 0]] so that elimination without row interchanges meets a zero pivot ("pivot")."""
    from oracle import henry as H
    J = np.zeros((20, ny, nx, S))
    if kind == "jacobian":
        pr = H.Problem(Lx=nx / 16.0, Ly=ny / 16.0)
        g = H.Grid(nx, ny, 12)
        th = draw_theta(74, S)
        for s in range(S):
            phi, K, u = H.sample_fields(pr, g, th[s])
            d = H.Discretisation(pr, g, phi, K, u)
            p0, _ = H.initial_state(pr, g)
            cc = rng.uniform(size=nx * ny)
            A = d.jacobian(p0 + 20.0 * rng.normal(size=nx * ny), cc).tocsr()
            for j in range(ny):
                for i in range(nx):
                    Pc = j * nx + i
                    for blk, (di, dj) in enumerate(((0, 0), (-1, 0), (1, 0), (0, -1), (0, 1))):
                        qi, qj = i + di, j + dj
                        if 0 <= qi < nx and 0 <= qj < ny:
                            Q = qj * nx + qi
                            for a in range(2):
                                for b in range(2):
                                    J[blk * 4 + a * 2 + b, j, i, s] = A[2 * Pc + a, 2 * Q + b]
    else:
        J[:] = rng.normal(size=J.shape)
        J[4:8, :, 0] = 0.0    # no west neighbour
        J[8:12, :, -1] = 0.0
        J[12:16, 0] = 0.0
        J[16:20, -1] = 0.0
        J[0:4, 0, 0] = np.array([0.0, 1.0, 1.0, 0.0])[:, None]
    return J, rng.normal(size=(2, ny, nx, S))


@pytest.mark.parametrize("kind", ["jacobian", "pivot"])
def test_coarse_solvers_against_numpy(hx, kind):
    import paper_2403_17018_amd as P
    rng = np.random.default_rng(20)
    S = 3
    for nx, ny in ((8, 4), (16, 8), (32, 16)):
        J, b = _coarse_case(rng, nx, ny, S, kind)
        g = P.grid(nx, ny, 1)
        for solver in ((0, 1, 2) if kind == "jacobian" else (1, 2)):
            if solver == 0 and ny > 16:
                continue
            for prec in (64, 32):
                for tr in (False, True):
                    x = _np(hx.coarse_solve(_cu(J), _cu(b), g, solver, prec, tr))
                    for s in range(S):
                        A = _blocks_to_sparse(J[..., s], nx, ny).toarray()
                        A = A.T if tr else A
                        bs = np.stack([b[0, ..., s].ravel(), b[1, ..., s].ravel()], axis=1).ravel()
                        xs = np.stack([x[0, ..., s].ravel(), x[1, ..., s].ravel()], axis=1).ravel()
                        ref = np.linalg.solve(A, bs)
                        # normwise backward error of the computed solution, and agreement with LAPACK
                        berr = np.abs(A @ xs - bs).max() / (np.abs(A).sum(axis=1).max() * np.abs(xs).max()
                                                            + np.abs(bs).max())
                        cond = np.linalg.cond(A, np.inf)
                        eps = 2.2e-16 if prec == 64 else 1.2e-7
                        assert berr <= 200 * eps, (nx, ny, solver, prec, tr, s, berr)
                        assert np.abs(xs - ref).max() <= 1000 * eps * cond * np.abs(ref).max(), \
                            (nx, ny, solver, prec, tr, s)


def test_named_configuration_32x16_dense_lu_matches_oracle(hx):
    """The 32x16 coarsest grid with the dense pivoted LU and the pivoted band LU (FP64 and FP32
    multigrid each) and with the banded LU, on a level-2 batch (128x64 cells: 3 grids) against
    the oracle."""
    import paper_2403_17018_amd as P
    th = draw_theta(75, 6, level=2)
    g = P.grid(128, 64, 30)
    T = 36000.0 * 30 / 192
    prob = P.problem(T=T)
    ref = oracle_batch(th, 128, 64, 30, dict(T=T))
    for solver, prec in ((1, 64), (1, 32), (2, 64), (2, 32), (0, 64)):
        o = P.solver_opts(coarse_nx=32, coarse_ny=16, coarse_solver=solver, mg_precision=prec)
        r = hx.solve(_cu(th), g, prob, o, want_c=True, want_p=True)
        assert r.nfailed == 0
        c = _sample_major(_np(r.c_T))
        p = _sample_major(_np(r.p_T))
        assert rel_inf(c, ref["c"]).max() <= 1e-8, (solver, prec)
        assert rel_inf(p, ref["p"]).max() <= 1e-8, (solver, prec)


def test_adjoint_with_dense_coarse_lu(hx):
    """The transposed dense and pivoted band solves inside the adjoint's transposed multigrid
    (64x32 cells, coarse 32x16): the gradient equals the one with the banded coarse solver to
    the solve tolerance."""
    import paper_2403_17018_amd as P
    th = draw_theta(76, 4, level=1)
    g = P.grid(64, 32, 8)
    prob = P.problem(T=6000.0)
    tight = dict(newton_tol=1e-13, krylov_rtol=1e-12, krylov_maxit=200, newton_maxit=60, krylov_rtol_adjoint=1e-12)
    out = []
    for solver, prec in ((0, 64), (1, 64), (1, 32), (2, 64), (2, 32)):
        o = P.solver_opts(coarse_nx=32, coarse_ny=16, coarse_solver=solver, mg_precision=prec, **tight)
        q, gr, st, nf = hx.adjoint(_cu(th), g, prob, o, checkpoint_every=3)
        assert nf == 0
        out.append(_np(gr))
    for gr in out[1:]:
        for s in range(4):
            assert np.abs(gr[s] - out[0][s]).max() <= 1e-9 * np.abs(out[0][s]).max(), s
