"""Ragged multi-level batching, hipGraph replay and the MLMC driver on the GPU."""
import numpy as np
import pytest
import torch

from henry_inputs import draw_theta
from tests.oracle_runs import oracle_batch, rel_inf

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hx():
    import paper_2403_17018_amd as P
    h = P.Henry(0)
    yield h
    h.close()


def _cu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_ragged_call_matches_separate_calls(hx):
    """Three batches, two on the same grid (merged inside the library), one on another grid
    (its own stream): each equals its separate solve to within the Newton tolerance (1e-9
    relative).  Merging changes iteration paths -- Jacobian refreshes, compaction and the
    Krylov half-step exit are decided per batch -- but not the discrete solution."""
    import paper_2403_17018_amd as P
    T = 7500.0
    prob = P.problem(T=T)
    a, b, c = draw_theta(31, 24), draw_theta(32, 40), draw_theta(33, 9)
    ga, gc = P.grid(32, 16, 10), P.grid(64, 32, 20)
    rr = hx.solve_ragged([(_cu(a), ga), (_cu(c), gc), (_cu(b), ga)], prob, want_p=True)
    for th, g, r in ((a, ga, rr[0]), (c, gc, rr[1]), (b, ga, rr[2])):
        s = hx.solve(_cu(th), g, prob, want_p=True)
        assert r.nfailed == 0 and s.nfailed == 0
        for x, y in ((r.c_T, s.c_T), (r.p_T, s.p_T)):
            x, y = x.cpu().numpy(), y.cpu().numpy()
            assert np.abs(x - y).max() <= 1e-9 * np.abs(y).max()
        assert np.allclose(r.qoi.cpu().numpy(), s.qoi.cpu().numpy(), rtol=1e-9, atol=0)


def test_same_grid_and_size_with_other_step_counts(hx):
    """Two batches on one grid with the same sample count but different step counts are solved
    concurrently in one call (one stream each): each must equal its own separate solve.  They
    share a workspace shape, so the library gives each its own instance."""
    import paper_2403_17018_amd as P
    prob = P.problem(T=7200.0)
    a, b = draw_theta(61, 16), draw_theta(62, 16)
    ga, gb = P.grid(32, 16, 8), P.grid(32, 16, 12)
    rr = hx.solve_ragged([(_cu(a), ga), (_cu(b), gb)], prob, P.solver_opts(use_graphs=1), want_p=True)
    for th, g, r in ((a, ga, rr[0]), (b, gb, rr[1])):
        s = hx.solve(_cu(th), g, prob, P.solver_opts(use_graphs=1), want_p=True)
        assert r.nfailed == 0 and s.nfailed == 0
        for x, y in ((r.c_T, s.c_T), (r.p_T, s.p_T)):
            x, y = x.cpu().numpy(), y.cpu().numpy()
            assert np.abs(x - y).max() <= 1e-9 * np.abs(y).max()


def test_graph_replay_is_bitwise_equal_to_eager(hx):
    """Each BiCGStab iteration replayed from a captured hipGraph, many replays with eager
    Newton/assembly work in between, against the eager launch sequence."""
    import paper_2403_17018_amd as P
    th = _cu(draw_theta(0, 16))
    for prec in (64, 32):
        for g in (P.level_grid(0), P.grid(64, 32, 12)):
            e = hx.solve(th, g, opts=P.solver_opts(mg_precision=prec, use_graphs=0), want_p=True)
            r = hx.solve(th, g, opts=P.solver_opts(mg_precision=prec, use_graphs=1), want_p=True)
            assert torch.equal(e.c_T, r.c_T) and torch.equal(e.p_T, r.p_T) and torch.equal(e.stats, r.stats)


def test_ragged_with_graphs_matches_oracle(hx):
    import paper_2403_17018_amd as P
    T = 6000.0
    a, b = draw_theta(41, 20), draw_theta(42, 6)
    ga, gb = P.grid(32, 16, 8), P.grid(64, 32, 16)
    rr = hx.solve_ragged([(_cu(a), ga), (_cu(b), gb)], P.problem(T=T), P.solver_opts(use_graphs=1, mg_precision=32))
    for th, g, r in ((a, ga, rr[0]), (b, gb, rr[1])):
        ref = oracle_batch(th, g.nx, g.ny, g.nsteps, dict(T=T))
        assert r.nfailed == 0
        c = r.c_T.permute(2, 0, 1).cpu().numpy()
        assert rel_inf(c, ref["c"]).max() <= 1e-8


def test_mlmc_run_matches_oracle_estimator(hx):
    """Levels 0..2 with coupled fine/coarse pairs in one ragged call; the estimate equals the
    oracle's estimator applied to oracle solves of the same samples."""
    import paper_2403_17018_amd as P
    from oracle import mlmc as M
    m = [24, 8, 4]
    thetas = [draw_theta(3, k, level=l) for l, k in enumerate(m)]
    est = P.mlmc_run(hx, [_cu(t) for t in thetas], [0, 1, 2], opts=P.solver_opts(use_graphs=1))
    assert est["nfailed"] == 0
    gf, gc, cf, cc = [], [], [], []
    for l, th in enumerate(thetas):
        nx, ny, ns = 32 << l, 16 << l, 48 << l
        f = oracle_batch(th, nx, ny, ns)
        gf.append(f["qoi"])
        cf.append(f["c"])
        if l > 0:
            c = oracle_batch(th, nx // 2, ny // 2, ns // 2)
            gc.append(c["qoi"])
            cc.append(c["c"])
        else:
            gc.append(None)
            cc.append(None)
    ref = M.estimate(gf, gc)
    assert est["mean"] == pytest.approx(ref["mean"], rel=1e-8)
    assert np.allclose(est["V"], ref["V"], rtol=1e-6, atol=1e-9 * ref["V"].max())
    assert est["rmse"] == pytest.approx(ref["rmse"], rel=1e-6)
    mf, vf = M.field_estimate(cf, cc)
    assert np.abs(est["mean_field"].cpu().numpy() - mf).max() <= 1e-8
    assert np.abs(est["var_field"].cpu().numpy() - vf).max() <= 1e-8


def test_autotune_returns_a_valid_faster_config(hx):
    """The tuner's choice solves to the same discrete solution as the defaults."""
    import paper_2403_17018_amd as P
    th = _cu(draw_theta(51, 48))
    g = P.grid(64, 32, 6)
    o, ms = hx.autotune(th, g)
    assert ms > 0 and o.coarse_nx in (8, 16) and o.nu_pre in (1, 2) and o.nu_post in (1, 2)
    assert o.red_blocks in (1024, 4096, 16384)
    a = hx.solve(th, g, opts=o, want_p=True)
    b = hx.solve(th, g, want_p=True)
    assert a.nfailed == 0 and b.nfailed == 0
    ca, cb = a.c_T.cpu().numpy(), b.c_T.cpu().numpy()
    assert np.abs(ca - cb).max() <= 1e-8 * np.abs(cb).max()


def _host_syncs(hx):
    return hx.profile_read()["host_sync"][0]


@pytest.mark.parametrize("prec", [64, 32])
def test_step_graphs_match_oracle_and_eager_series(hx, prec):
    """Steps whose first Newton iteration is replayed from one captured graph (device-side
    control, one host read per step): c and p at T against the oracle (1e-8), and the salt
    masses after every step against the eager solve, so each of the replays -- with eager
    continuation iterations, balance kernels and host reads between them -- is checked; the
    replayed path needs fewer host round trips."""
    import paper_2403_17018_amd as P
    th = draw_theta(0, 16)
    g = P.level_grid(0)
    ref = oracle_batch(th, g.nx, g.ny, g.nsteps)
    out = {}
    for sg in (0, 1):
        n0 = _host_syncs(hx)
        r = hx.solve(_cu(th), g, opts=P.solver_opts(mg_precision=prec, step_graphs=sg), want_p=True,
                     want_series=True)
        torch.cuda.synchronize()
        out[sg] = (r, _host_syncs(hx) - n0)
        assert r.nfailed == 0
        c = r.c_T.permute(2, 0, 1).cpu().numpy()
        p = r.p_T.permute(2, 0, 1).cpu().numpy()
        assert rel_inf(c, ref["c"]).max() <= 1e-8 and rel_inf(p, ref["p"]).max() <= 1e-8, sg
    se, sg_ = out[0][0].series.cpu().numpy(), out[1][0].series.cpu().numpy()   # [nsteps, 17, S]
    mass = [0] + list(range(2, 17))                                               # Q_S and the box masses
    for k in range(g.nsteps):
        a, b = se[k, mass], sg_[k, mass]
        assert np.abs(a - b).max() <= 1e-8 * np.abs(a).max(), k
    assert out[1][1] < out[0][1], (out[1][1], out[0][1])


def test_ragged_threads_sequential_equals_concurrent(hx):
    """The grids of a ragged call run from the calling thread one after another give bitwise
    the results of one host thread per grid."""
    import paper_2403_17018_amd as P
    prob = P.problem(T=6000.0)
    a, b = draw_theta(63, 12), draw_theta(64, 5)
    items = [(_cu(a), P.grid(32, 16, 8)), (_cu(b), P.grid(64, 32, 16))]
    r0 = hx.solve_ragged(items, prob, P.solver_opts(ragged_threads=0), want_p=True)
    r1 = hx.solve_ragged(items, prob, P.solver_opts(ragged_threads=1), want_p=True)
    for x, y in zip(r0, r1):
        assert torch.equal(x.c_T, y.c_T) and torch.equal(x.p_T, y.p_T) and torch.equal(x.stats, y.stats)
