"""The library's kernel-class profiler (henry_profile, henry_profile_read): every timed class
of a solve reports launches, units and event time, and turning the profiler on leaves every
result bit for bit unchanged on the same launch path (graphs, which the profiler skips, off)."""
import numpy as np
import pytest
import torch

from henry_inputs import draw_theta

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hx():
    import paper_2403_17018_amd as P
    h = P.Henry(0)
    yield h
    h.close()


def _cu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _profiled(hx, run):
    hx.profile(True)
    r = run()
    torch.cuda.synchronize()
    prof = hx.profile_read()
    hx.profile(False)
    return r, prof


@pytest.mark.parametrize("opts,coarse", [
    (dict(), ("band_factor", "band_solve")),
    (dict(mg_precision=32), ("band_factor", "band_solve")),
    (dict(coarse_nx=16, coarse_ny=8, coarse_solver=1), ("dense_factor", "dense_solve")),
    (dict(coarse_nx=16, coarse_ny=8, coarse_solver=2), ("band_factor", "band_solve")),
])
def test_cell_centred_classes(hx, opts, coarse):
    import paper_2403_17018_amd as P
    th = _cu(draw_theta(92, 80, level=0))
    g = P.grid(32, 16, 12)
    # whole-step graphs are skipped while profiling (their launches cannot be timed), which
    # changes the control path: compare both runs without them
    o = P.solver_opts(step_graphs=0, **opts)
    a = hx.solve(th, g, opts=o, want_c=True, want_p=True)
    b, prof = _profiled(hx, lambda: hx.solve(th, g, opts=o, want_c=True, want_p=True))
    assert torch.equal(a.c_T, b.c_T) and torch.equal(a.p_T, b.p_T) and torch.equal(a.stats, b.stats)
    for cls in ("assemble", "gs", "spmv", "restrict", "prolong") + coarse:
        n, units, ms = prof[cls]
        assert n > 0 and units > 0 and ms > 0.0, cls
        assert ms / n < 50.0, cls            # one kernel on a 32x16 grid: far below 50 ms
    n_as, u_as, _ = prof["assemble"]
    assert u_as == n_as * 32 * 16 * 80       # cell-samples of the fine grid per assembly
    n_gs, u_gs, _ = prof["gs"]
    assert u_gs == n_gs * 16 * 16 * 80       # one colour: half the cells per pass
    assert prof["host_sync"][0] > 0


def test_vertex_centred_classes(hx):
    import paper_2403_17018_amd as P
    th = _cu(draw_theta(93, 40))
    g = P.vc_level_grid(0)
    o = P.solver_opts(krylov_maxit=300)
    a = hx.vc_solve(th, g, P.paper_problem(), o, want_c=True, want_p=True)
    b, prof = _profiled(hx, lambda: hx.vc_solve(th, g, P.paper_problem(), o, want_c=True, want_p=True))
    assert torch.equal(a.c_T, b.c_T) and torch.equal(a.p_T, b.p_T) and torch.equal(a.stats, b.stats)
    nv = 17 * 9
    n_as, u_as, ms_as = prof["assemble"]
    assert n_as > 0 and u_as == n_as * nv * 40 and ms_as > 0.0
    n_sp, u_sp, ms_sp = prof["spmv"]
    assert n_sp > 0 and u_sp == n_sp * nv * 40 and ms_sp > 0.0
    n_gs, u_gs, ms_gs = prof["gs"]
    # four colours per sweep: 9*5, 8*5, 9*4 and 8*4 vertices, equal numbers of each colour pass
    assert n_gs % 4 == 0 and u_gs == (n_gs // 4) * (45 + 40 + 36 + 32) * 40 and ms_gs > 0.0
    assert prof["host_sync"][0] > 0
