"""mlmc_estimate_noalloc (the allocation-free estimator) against mlmc_estimate, both through
the C ABI on the same device inputs: two calls in a row, the second with a smaller input
(fewer levels and samples), must give bitwise the same scalars and fields; a request beyond
the stated workspace is refused before any work."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hx():
    import paper_2403_17018_amd as P
    h = P.Henry(0)
    yield h
    h.close()


def _inputs(L, m, seed):
    import paper_2403_17018_amd as P
    rng = np.random.default_rng(seed)
    grids = [P.level_grid(l) for l in range(L + 1)]
    cu = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    gf = [cu(300.0 + rng.normal(size=m[l])) for l in range(L + 1)]
    gc = [None] + [cu(gf[l].cpu().numpy() - 2.0 ** -l + 0.1 * rng.normal(size=m[l])) for l in range(1, L + 1)]
    cf = [cu(rng.uniform(size=(g.ny, g.nx, m[l]))) for l, g in enumerate(grids)]
    cc = [None] + [cu(rng.uniform(size=(grids[l - 1].ny, grids[l - 1].nx, m[l]))) for l in range(1, L + 1)]
    return grids, gf, gc, cf, cc


def _same(a, b):
    assert a["mean"] == b["mean"] and a["var_of_estimator"] == b["var_of_estimator"] and a["rmse"] == b["rmse"]
    assert a["V"] == b["V"]
    assert torch.equal(a["mean_field"], b["mean_field"]) and torch.equal(a["var_field"], b["var_field"])


def test_noalloc_estimator_equals_allocating_one(hx):
    for L, m, seed in ((4, [64, 32, 16, 8, 4], 1), (2, [16, 8, 4], 2)):   # the second call is smaller
        grids, gf, gc, cf, cc = _inputs(L, m, seed)
        a = hx.mlmc_estimate(grids, gf, gc, cf, cc, alpha=1.0)
        b = hx.mlmc_estimate(grids, gf, gc, cf, cc, alpha=1.0, noalloc=True)
        torch.cuda.synchronize()
        print(f"L={L} m={m}: mean {a['mean']!r} rmse {a['rmse']!r}", flush=True)
        _same(a, b)
        s = hx.mlmc_estimate(grids, gf, gc, alpha=1.5, noalloc=True)    # scalars only
        r = hx.mlmc_estimate(grids, gf, gc, alpha=1.5)
        assert s["mean"] == r["mean"] and s["rmse"] == r["rmse"] and s["V"] == r["V"]


def test_noalloc_refuses_more_than_its_workspace(hx):
    import paper_2403_17018_amd as P
    L, m = 6, [2] * 7                                                      # finest grid 2048 x 1024
    grids, gf, gc, cf, cc = _inputs(L, m, 3)
    with pytest.raises(P.HenryError) as e:
        hx.mlmc_estimate(grids, gf, gc, cf, cc, noalloc=True)
    assert e.value.code == -1
    a = hx.mlmc_estimate(grids[:3], gf[:3], gc[:3], cf[:3], cc[:3])       # the context is still usable
    b = hx.mlmc_estimate(grids[:3], gf[:3], gc[:3], cf[:3], cc[:3], noalloc=True)
    _same(a, b)
