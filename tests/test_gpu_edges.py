"""Edge cases of the batched solve against the oracle: one sample, a batch one past a full
wavefront of samples (a tail block of one sample), batch sizes that select the multigrid's
wide launches (several samples per thread) against one sample per thread, an odd number of
rows (the hierarchy stops at once and the banded LU solves the whole grid), and empty or
invalid batches."""
import numpy as np
import pytest
import torch

from henry_inputs import draw_theta
from tests.oracle_runs import oracle_batch, rel_inf

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


@pytest.mark.parametrize("S,pick", [(1, [0]), (65, [0, 63, 64])])
def test_batch_sizes_around_a_wavefront(hx, S, pick):
    """64 samples fill one wavefront per cell; S = 65 leaves a one-sample tail block."""
    import paper_2403_17018_amd as P
    th = draw_theta(8, S, level=1)
    g = P.grid(64, 32, 24)
    kw = dict(T=9000.0)
    r = hx.solve(_cuda(th), g, P.problem(**kw), want_c=True, want_p=True)
    assert r.nfailed == 0
    c = r.c_T.permute(2, 0, 1).cpu().numpy()[pick]
    p = r.p_T.permute(2, 0, 1).cpu().numpy()[pick]
    ref = oracle_batch(th[pick], g.nx, g.ny, g.nsteps, kw)
    assert rel_inf(c, ref["c"]).max() <= TOL
    assert rel_inf(p, ref["p"]).max() <= TOL
    assert np.abs(r.qoi.cpu().numpy()[pick] - ref["qoi"]).max() <= TOL * np.abs(ref["qoi"]).max()


@pytest.mark.parametrize("prec", [64, 32])
@pytest.mark.parametrize("S", [256, 320, 600])
def test_wide_stencil_kernels_match_one_sample_per_thread(hx, prec, S):
    """A batch of S runs the multigrid's smoother, restriction and prolongation with several
    adjacent samples per thread (2 in FP64, 4 in FP32; rows of 64 threads at S = 256, of 32
    or 16 at S = 320 and of 64 or 32 at S = 600, so that no more lanes idle than with one
    sample per thread); the same samples in a batch of S - 1 (not a multiple of the width)
    run one sample per thread.  Samples are independent, so each must come out the same to
    rounding, and (at S = 256) both must match the oracle."""
    import paper_2403_17018_amd as P
    th = draw_theta(10, S, level=1)
    g = P.grid(64, 32, 16)
    kw = dict(T=6000.0)
    pick = [0, 127, 254]
    ref = oracle_batch(th[pick], g.nx, g.ny, g.nsteps, kw) if S == 256 else None
    for opts in (P.solver_opts(mg_precision=prec, fuse_prolong=0), P.solver_opts(mg_precision=prec)):
        a = hx.solve(_cuda(th), g, P.problem(**kw), opts, want_c=True, want_p=True)
        b = hx.solve(_cuda(th[:S - 1]), g, P.problem(**kw), opts, want_c=True, want_p=True)
        assert a.nfailed == 0 and b.nfailed == 0
        for fa, fb in ((a.c_T, b.c_T), (a.p_T, b.p_T)):
            fa = fa.permute(2, 0, 1).cpu().numpy()[:S - 1]
            fb = fb.permute(2, 0, 1).cpu().numpy()
            assert rel_inf(fa, fb).max() <= 1e-12
        if ref is not None:
            c = a.c_T.permute(2, 0, 1).cpu().numpy()[pick]
            assert rel_inf(c, ref["c"]).max() <= TOL


def test_odd_rows_single_level(hx):
    """34 x 17 cells: 17 rows cannot be halved, so the whole grid is the banded-LU level."""
    import paper_2403_17018_amd as P
    th = draw_theta(9, 6)
    g = P.grid(34, 17, 10)
    kw = dict(T=7500.0)
    for prec in (64, 32):
        r = hx.solve(_cuda(th), g, P.problem(**kw), P.solver_opts(mg_precision=prec), want_c=True)
        assert r.nfailed == 0
        ref = oracle_batch(th, g.nx, g.ny, g.nsteps, kw)
        assert rel_inf(r.c_T.permute(2, 0, 1).cpu().numpy(), ref["c"]).max() <= TOL, prec


def test_empty_and_invalid_batches(hx):
    import paper_2403_17018_amd as P
    assert hx.solve_ragged([]) == []
    empty = torch.empty((0, 13), dtype=torch.float64, device="cuda")
    with pytest.raises(P.HenryError) as e:
        hx.solve(empty, P.level_grid(0))
    assert e.value.code == -1
    th = _cuda(draw_theta(0, 2))
    with pytest.raises(P.HenryError):
        hx.solve(th, P.grid(1, 1, 4))          # fewer than 2 cells per direction
    with pytest.raises(P.HenryError):
        hx.solve(th, P.grid(32, 16, 0))        # no time steps
    with pytest.raises(P.HenryError):
        hx.solve(th, P.level_grid(0), P.problem(field_model=2))


def test_out_of_memory_is_an_error_not_a_crash(hx):
    """A batch whose workspace cannot fit in device memory (level 4, two million samples:
    terabytes per field) is refused with HENRY_ENOMEM; the context stays usable."""
    import paper_2403_17018_amd as P
    th = torch.zeros((2_000_000, 13), dtype=torch.float64, device="cuda")
    with pytest.raises(P.HenryError) as e:
        hx.solve(th, P.level_grid(4), want_c=False)
    assert e.value.code == -3
    del th
    r = hx.solve(_cuda(draw_theta(0, 2)), P.grid(32, 16, 2), want_c=True)
    assert r.nfailed == 0
