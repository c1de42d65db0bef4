"""Time-resolved QoIs (section 5: Q_S, Q_FW and the 15 box masses after every step) from
the GPU solve against the oracle's, for the KL workload model and the paper's own model.

Tolerance: the solve's bound |c_gpu - c_oracle| <= 1e-8 max|c| (max|c| <= 1) carried through
each integral: a salt mass over a region of area A may differ by 1e-8 (rho0 + 2 drho) A
(the derivative of c rho(c) is at most rho0 + 2 drho); the fresh-water area Q_FW counts cells
by c <= 0.012178, so it may differ by the area of the cells whose oracle c lies within 1e-8
of the threshold."""
import math

import numpy as np
import pytest
import torch

from henry_inputs import draw_theta
from tests.oracle_runs import oracle_batch

pytestmark = pytest.mark.gpu
TOL = 1e-8


@pytest.fixture(scope="module")
def hx():
    import paper_2403_17018_amd as P
    h = P.Henry(0)
    yield h
    h.close()


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("model", ["kl", "paper"])
def test_series_match_oracle(hx, model):
    import paper_2403_17018_amd as P
    if model == "kl":
        th, g, prob, okw = draw_theta(3, 8), P.level_grid(0), P.problem(), {}
    else:
        th, g = draw_theta(5, 8, level=1), P.level_grid(1)
        prob = P.paper_problem()
        okw = dict(field_model="paper", q_in_amp=0.5, recharge_omega=math.pi / 40.0, T=6016.0)
    r = hx.solve(_cuda(th), g, prob, want_series=True)
    assert r.nfailed == 0
    s = r.series.permute(2, 0, 1).cpu().numpy()          # [S, nsteps, 17]
    ref = oracle_batch(th, g.nx, g.ny, g.nsteps, okw, series=True)
    z = ref["series"]
    assert s.shape == z.shape == (8, g.nsteps, 17)
    area = [2.0, None] + [0.2 * 0.15] * 5 + [0.2 * 0.2] * 10
    for q in [0] + list(range(2, 17)):
        assert (np.abs(s[:, :, q] - z[:, :, q]) <= TOL * (1000.0 + 2 * 25.0) * area[q]).all(), q
    assert (np.abs(s[:, :, 1] - z[:, :, 1]) <= ref["fw_ambiguous"] + 1e-12).all()
    # the last step's whole-domain salt mass bounds the x > 1 QoI
    assert (s[:, -1, 0] >= r.qoi.cpu().numpy()).all()


def test_series_of_merged_batches_equal_separate_calls(hx):
    """Two batches on one grid are merged into one plan; their series are scattered back."""
    import paper_2403_17018_amd as P
    th = _cuda(draw_theta(3, 12))
    g = P.grid(32, 16, 6)
    a, b = hx.solve_ragged([(th[:5].contiguous(), g), (th[5:].contiguous(), g)], want_series=True)
    whole = hx.solve(th, g, want_series=True)
    assert torch.equal(torch.cat([a.series, b.series], dim=2), whole.series)


def test_series_estimator_matches_oracle(hx):
    """mlmc_estimate_series on random series of three levels (r_l = 4, 8, 16 steps, 3 QoIs)."""
    import paper_2403_17018_amd as P
    from oracle import mlmc as M
    rng = np.random.default_rng(1)
    m = [33, 10, 5]
    r = [4, 8, 16]
    sf = [rng.normal(size=(r[l], 3, m[l])) + 2.0 for l in range(3)]
    sc = [None] + [sf[l][::2] * 0.0 + rng.normal(size=(r[l - 1], 3, m[l])) + 2.0 for l in (1, 2)]
    grids = [P.grid(8 << l, 4 << l, r[l]) for l in range(3)]
    out = hx.mlmc_estimate_series(grids, [_cuda(a) for a in sf], [None] + [_cuda(a) for a in sc[1:]])
    ref = M.estimate_series([np.moveaxis(a, -1, 0) for a in sf], [None] + [np.moveaxis(a, -1, 0) for a in sc[1:]])
    for k in ("mean", "var_of_estimator", "Ymean", "V"):
        np.testing.assert_allclose(out[k].cpu().numpy(), ref[k], rtol=1e-12, atol=1e-14)


def test_adaptive_mlmc_plan_and_estimate(hx):
    """The adaptive driver: its plan is the oracle's plan of the pilot statistics it measured,
    and its estimate is the oracle's estimator of the production QoIs."""
    import paper_2403_17018_amd as P
    from oracle import mlmc as M

    def sampler(level, n, first):
        return _cuda(draw_theta(11, n, level=level, first_sample=first))

    est = P.mlmc_adaptive(hx, sampler, eps=0.05, pilot_levels=2, pilot_samples=24, max_level=3)
    assert est["nfailed"] == 0
    pl, pp = est["plan"], est["pilot"]
    ref = M.plan(pp["Ymean_abs"], pp["V"], pp["s"], 0.05, pp["E0"], 3)
    assert pl["L"] == ref["L"] and pl["m"] == ref["m"]
    res = est["results"]
    gf, gc, k = [], [], 0
    for l in range(pl["L"] + 1):
        gf.append(res[k].qoi.cpu().numpy())
        gc.append(res[k + 1].qoi.cpu().numpy() if l > 0 else None)
        k += 2 if l > 0 else 1
    e = M.estimate(gf, gc, alpha=pl["alpha"])
    assert est["mean"] == pytest.approx(e["mean"], rel=1e-12)
    assert est["rmse"] == pytest.approx(e["rmse"], rel=1e-10)
