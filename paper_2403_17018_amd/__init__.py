"""Batched stochastic Henry problem and MLMC on AMD MI355X (gfx950).

Thin Python binding of libhenry (include/henry.h).  Every step of the solve runs in
the library's HIP kernels; this module only marshals torch tensors (device memory)
and the current torch stream into the C ABI.  There is no CPU fallback: without the
built libhenry.so every call raises.
"""
from __future__ import annotations

import ctypes as C
import math
import dataclasses

import torch

from . import _lib as L
from ._lib import henry_batch, henry_grid, henry_problem, henry_solver_opts

__all__ = ["Henry", "HenryError", "problem", "paper_problem", "solver_opts", "grid", "level_grid", "optimal_samples",
           "SolveResult", "mlmc_run", "mlmc_plan", "mlmc_adaptive", "SaltMassQoI", "salt_mass_qoi", "vc_level_grid",
           "mlmc_run_vc"]

STATUS = {0: "ok", 1: "newton", 2: "krylov", 3: "nonfinite", 4: "range"}


class HenryError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libhenry error {code}: {msg}")
        self.code = code


def problem(**kw) -> henry_problem:
    """henry_problem with the library's defaults, fields overridden by keyword."""
    p = henry_problem()
    L.load().henry_problem_default(C.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


def paper_problem(**kw) -> henry_problem:
    """The paper's own stochastic model (section 4): two-layer multiscale porosity with
    xi_1 = theta[0], xi_2 = theta[1], Kozeny-Carman permeability, recharge
    6.6e-5 (1 + 0.5 xi_3)(1 + sin(pi t/40)) m/s with xi_3 = theta[12], T = 6016 s."""
    d = dict(field_model=1, q_in_amp=0.5, recharge_omega=math.pi / 40.0, T=6016.0)
    d.update(kw)
    return problem(**d)


def solver_opts(**kw) -> henry_solver_opts:
    o = henry_solver_opts()
    L.load().henry_solver_opts_default(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


def grid(nx: int, ny: int, nsteps: int) -> henry_grid:
    return henry_grid(nx, ny, nsteps)


def vc_level_grid(level: int) -> henry_grid:
    """Level l of the paper's Table 2 for the vertex-centred discretisation: 16*4^l x 8*4^l
    elements ((16*4^l + 1)(8*4^l + 1) vertices), 94*4^l implicit-Euler steps."""
    return henry_grid(16 * 4 ** level, 8 * 4 ** level, 94 * 4 ** level)


def level_grid(level: int) -> henry_grid:
    """MLMC level l: 32*2^l x 16*2^l cells, 48*2^l implicit-Euler steps."""
    return henry_grid(32 << level, 16 << level, 48 << level)


@dataclasses.dataclass
class SolveResult:
    c_T: torch.Tensor | None      # [ny, nx, S]
    p_T: torch.Tensor | None
    qoi: torch.Tensor             # [S]
    status: torch.Tensor          # [S] int32
    stats: torch.Tensor           # [S, 4]
    nfailed: int
    series: torch.Tensor | None = None   # [nsteps, 17, S]: Q_S, Q_FW, Q_1..Q_15 after every step


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _check_theta(theta, device):
    if not (isinstance(theta, torch.Tensor) and theta.dtype == torch.float64 and theta.is_cuda):
        raise TypeError("theta must be a float64 CUDA tensor")
    if theta.dim() != 2 or theta.shape[1] != 13 or not theta.is_contiguous():
        raise ValueError("theta must be contiguous [S, 13]")
    if theta.device != device:
        raise ValueError("theta is on another device")


class Henry:
    """A libhenry context bound to one device and one HIP stream."""

    def __init__(self, device: int = 0, stream: torch.cuda.Stream | None = None):
        self._lib = L.load()
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        rc = self._lib.henry_ctx_create(C.byref(h), device, C.c_void_p(self.stream.cuda_stream))
        if rc != 0:
            raise HenryError(rc, "henry_ctx_create failed")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._lib.henry_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc < 0:
            raise HenryError(rc, self._lib.henry_last_error(self._h).decode())
        return rc

    def sample_fields(self, theta, g: henry_grid, prob: henry_problem | None = None):
        _check_theta(theta, self.device)
        S = theta.shape[0]
        prob = prob or problem()
        kw = dict(dtype=torch.float64, device=self.device)
        phi = torch.empty((g.ny, g.nx, S), **kw)
        K = torch.empty((g.ny, g.nx, S), **kw)
        q = torch.empty((S,), **kw)
        self._check(self._lib.henry_sample_fields(self._h, C.byref(prob), g, S, _ptr(theta), _ptr(phi), _ptr(K), _ptr(q)))
        return phi, K, q

    def solve_ragged(self, items, prob: henry_problem | None = None, opts: henry_solver_opts | None = None,
                     want_c: bool = True, want_p: bool = False, want_series: bool = False):
        """items: list of (theta [S,13], henry_grid).  One call; returns a list of SolveResult."""
        prob = prob or problem()
        opts = opts or solver_opts()
        kw = dict(dtype=torch.float64, device=self.device)
        arr = (henry_batch * len(items))()
        res = []
        for b, (theta, g) in enumerate(items):
            _check_theta(theta, self.device)
            S = theta.shape[0]
            r = SolveResult(
                c_T=torch.empty((g.ny, g.nx, S), **kw) if want_c else None,
                p_T=torch.empty((g.ny, g.nx, S), **kw) if want_p else None,
                qoi=torch.empty((S,), **kw),
                status=torch.empty((S,), dtype=torch.int32, device=self.device),
                stats=torch.empty((S, 4), **kw), nfailed=0,
                series=torch.empty((g.nsteps, L.NSERIES, S), **kw) if want_series else None)
            arr[b] = henry_batch(g, S, theta.data_ptr(), _ptr(r.c_T), _ptr(r.p_T), _ptr(r.qoi), _ptr(r.status),
                                 _ptr(r.stats), _ptr(r.series))
            res.append(r)
        rc = self._check(self._lib.henry_solve_batch(self._h, C.byref(prob), C.byref(opts), arr, len(items)))
        for r in res:
            r.nfailed = int((r.status != 0).sum().item())
        assert sum(r.nfailed for r in res) == rc
        return res

    def solve(self, theta, g: henry_grid, prob=None, opts=None, want_c=True, want_p=False,
              want_series=False) -> SolveResult:
        return self.solve_ragged([(theta, g)], prob, opts, want_c, want_p, want_series)[0]

    def adjoint(self, theta, g: henry_grid, prob=None, opts=None, checkpoint_every: int = 32):
        """(qoi [S], dqoi/dtheta [S,13], status [S], nfailed)."""
        _check_theta(theta, self.device)
        prob = prob or problem()
        opts = opts or solver_opts()
        S = theta.shape[0]
        kw = dict(dtype=torch.float64, device=self.device)
        q = torch.empty((S,), **kw)
        gr = torch.empty((S, 13), **kw)
        st = torch.empty((S,), dtype=torch.int32, device=self.device)
        rc = self._check(self._lib.henry_adjoint_batch(self._h, C.byref(prob), C.byref(opts), g, S, _ptr(theta),
                                                       checkpoint_every, _ptr(q), _ptr(gr), _ptr(st)))
        return q, gr, st, rc

    def mlmc_estimate(self, grids, g_fine, g_coarse, c_fine=None, c_coarse=None, alpha: float = 1.0,
                      noalloc: bool = False, out=None):
        """Telescoping MLMC estimate over levels 0..L (device reductions).

        g_fine[l], g_coarse[l] (None for l = 0): float64 CUDA tensors [m_l];
        c_fine[l]: [ny_l, nx_l, m_l]; c_coarse[l]: [ny_{l-1}, nx_{l-1}, m_l] (None for l = 0).
        noalloc: call mlmc_estimate_noalloc (the library allocates nothing); out: optional
        (mean_field, var_field) tensors [ny_L, nx_L] to write instead of new ones.
        """
        Lv = len(g_fine) - 1
        m = (C.c_int * (Lv + 1))(*[int(t.numel()) for t in g_fine])
        gr = (henry_grid * (Lv + 1))(*grids)
        vp = C.c_void_p
        gf = (vp * (Lv + 1))(*[t.data_ptr() for t in g_fine])
        gc = (vp * (Lv + 1))(*[0 if t is None else t.data_ptr() for t in g_coarse])
        cf = cc = None
        mean_f = var_f = None
        if c_fine is not None:
            cf = (vp * (Lv + 1))(*[t.data_ptr() for t in c_fine])
            cc = (vp * (Lv + 1))(*[0 if t is None else t.data_ptr() for t in c_coarse])
            gL = grids[-1]
            if out is not None:
                mean_f, var_f = out
            else:
                mean_f = torch.empty((gL.ny, gL.nx), dtype=torch.float64, device=self.device)
                var_f = torch.empty_like(mean_f)
        mean, var, rmse = C.c_double(), C.c_double(), C.c_double()
        V = (C.c_double * (Lv + 1))()
        fn = self._lib.mlmc_estimate_noalloc if noalloc else self._lib.mlmc_estimate
        self._check(fn(self._h, Lv, m, gr, gf, gc, cf, cc, alpha, C.byref(mean), C.byref(var), C.byref(rmse), V,
                       _ptr(mean_f), _ptr(var_f)))
        return dict(mean=mean.value, var_of_estimator=var.value, rmse=rmse.value, V=list(V), mean_field=mean_f,
                    var_field=var_f)


    def mlmc_estimate_series(self, grids, s_fine, s_coarse):
        """Time-resolved MLMC (device reductions): s_fine[l] [r_l, nq, m_l], s_coarse[l]
        [r_{l-1}, nq, m_l] (None for l = 0), every r_l a multiple of r_0.  Returns dict of
        device tensors mean, var_of_estimator [r_0, nq] and Ymean, V [L+1, r_0, nq] at the
        common times (k + 1) T / r_0."""
        Lv = len(s_fine) - 1
        r0, nq = int(s_fine[0].shape[0]), int(s_fine[0].shape[1])
        for l, t in enumerate(s_fine):
            if not (t.dtype == torch.float64 and t.is_cuda and t.is_contiguous() and t.dim() == 3):
                raise TypeError("series must be contiguous float64 CUDA tensors [r, nq, m]")
            if l > 0 and (s_coarse[l] is None or s_coarse[l].shape[1:] != (nq, t.shape[2])):
                raise ValueError(f"level {l}: coarse series shape")
        m = (C.c_int * (Lv + 1))(*[int(t.shape[2]) for t in s_fine])
        ga = (henry_grid * (Lv + 1))(*grids)
        f = (C.c_void_p * (Lv + 1))(*[t.data_ptr() for t in s_fine])
        c = (C.c_void_p * (Lv + 1))(*[None if t is None else t.data_ptr() for t in s_coarse])
        kw = dict(dtype=torch.float64, device=self.device)
        out = dict(mean=torch.empty((r0, nq), **kw), var_of_estimator=torch.empty((r0, nq), **kw),
                   Ymean=torch.empty((Lv + 1, r0, nq), **kw), V=torch.empty((Lv + 1, r0, nq), **kw))
        self._check(self._lib.mlmc_estimate_series(self._h, Lv, m, ga, nq, f, c, _ptr(out["mean"]),
                                                   _ptr(out["var_of_estimator"]), _ptr(out["Ymean"]), _ptr(out["V"])))
        return out

    # kernel-level calls (single launches of the solve's kernels; tests and diagnostics)
    def _f64(self, t, shape, name):
        if not (isinstance(t, torch.Tensor) and t.dtype == torch.float64 and t.is_cuda and t.is_contiguous()
                and t.device == self.device and tuple(t.shape) == tuple(shape)):
            raise ValueError(f"{name} must be a contiguous float64 CUDA tensor of shape {tuple(shape)}")

    def assemble(self, theta, g: henry_grid, p, c, c_old, step: int, prob=None):
        """(R [2, ny, nx, S], J [20, ny, nx, S]) of implicit-Euler step `step` at (p, c)."""
        _check_theta(theta, self.device)
        S = theta.shape[0]
        for t, nm in ((p, "p"), (c, "c"), (c_old, "c_old")):
            self._f64(t, (g.ny, g.nx, S), nm)
        kw = dict(dtype=torch.float64, device=self.device)
        R = torch.empty((2, g.ny, g.nx, S), **kw)
        J = torch.empty((20, g.ny, g.nx, S), **kw)
        self._check(self._lib.henry_assemble(self._h, C.byref(prob or problem()), g, S, _ptr(theta), _ptr(p), _ptr(c),
                                             _ptr(c_old), step, _ptr(R), _ptr(J)))
        return R, J

    def vc_solve(self, theta, g: henry_grid, prob=None, opts=None, want_c=True, want_p=False):
        """The paper's vertex-centred discretisation on g.nx x g.ny elements (henry_vc_solve):
        SolveResult with c_T, p_T [ny+1, nx+1, S] at the vertices and stats [S, 2] (Newton,
        BiCGStab iterations)."""
        _check_theta(theta, self.device)
        S = theta.shape[0]
        kw = dict(dtype=torch.float64, device=self.device)
        r = SolveResult(c_T=torch.empty((g.ny + 1, g.nx + 1, S), **kw) if want_c else None,
                        p_T=torch.empty((g.ny + 1, g.nx + 1, S), **kw) if want_p else None,
                        qoi=torch.empty((S,), **kw), status=torch.zeros((S,), dtype=torch.int32, device=self.device),
                        stats=torch.zeros((S, 2), **kw), nfailed=0)
        rc = self._lib.henry_vc_solve(self._h, C.byref(prob or problem()), C.byref(opts or solver_opts()), g, S,
                                      _ptr(theta), _ptr(r.c_T), _ptr(r.p_T), _ptr(r.qoi), _ptr(r.status), _ptr(r.stats))
        self._check(rc)
        r.nfailed = rc
        return r

    def vc_solve_batch(self, items, prob=None, opts=None, want_c=True, want_p=False):
        """items: list of (theta [S,13], henry_grid) for the vertex-centred discretisation, solved
        in one call (henry_vc_solve_batch: each batch on its own stream and host thread).
        Returns a list of SolveResult as vc_solve gives."""
        kw = dict(dtype=torch.float64, device=self.device)
        arr = (henry_batch * len(items))()
        res = []
        for b, (theta, g) in enumerate(items):
            _check_theta(theta, self.device)
            S = theta.shape[0]
            r = SolveResult(c_T=torch.empty((g.ny + 1, g.nx + 1, S), **kw) if want_c else None,
                            p_T=torch.empty((g.ny + 1, g.nx + 1, S), **kw) if want_p else None,
                            qoi=torch.empty((S,), **kw), status=torch.zeros((S,), dtype=torch.int32, device=self.device),
                            stats=torch.zeros((S, 2), **kw), nfailed=0)
            arr[b] = henry_batch(g, S, theta.data_ptr(), _ptr(r.c_T), _ptr(r.p_T), _ptr(r.qoi), _ptr(r.status),
                                 _ptr(r.stats), None)
            res.append(r)
        rc = self._check(self._lib.henry_vc_solve_batch(self._h, C.byref(prob or problem()),
                                                        C.byref(opts or solver_opts()), arr, len(items)))
        for r in res:
            r.nfailed = int((r.status != 0).sum().item())
        assert sum(r.nfailed for r in res) == rc
        return res

    def vc_assemble(self, theta, g: henry_grid, p, c, c_old, step: int, prob=None):
        """(R [2, ny+1, nx+1, S], J [36, ny+1, nx+1, S]) of the vertex-centred step `step`."""
        _check_theta(theta, self.device)
        S = theta.shape[0]
        for t, nm in ((p, "p"), (c, "c"), (c_old, "c_old")):
            self._f64(t, (g.ny + 1, g.nx + 1, S), nm)
        kw = dict(dtype=torch.float64, device=self.device)
        R = torch.empty((2, g.ny + 1, g.nx + 1, S), **kw)
        J = torch.empty((36, g.ny + 1, g.nx + 1, S), **kw)
        self._check(self._lib.henry_vc_assemble(self._h, C.byref(prob or problem()), g, S, _ptr(theta), _ptr(p),
                                                _ptr(c), _ptr(c_old), step, _ptr(R), _ptr(J)))
        return R, J

    def jacobian_apply(self, J, x, g: henry_grid, transpose: bool = False):
        S = x.shape[-1]
        self._f64(J, (20, g.ny, g.nx, S), "J")
        self._f64(x, (2, g.ny, g.nx, S), "x")
        y = torch.empty_like(x)
        self._check(self._lib.henry_jacobian_apply(self._h, g, S, _ptr(J), _ptr(x), _ptr(y), int(transpose)))
        return y

    def gs_pass(self, J, b, x, g: henry_grid, colour: int, transpose: bool = False):
        """One red (0) or black (1) Gauss-Seidel pass, in place on x."""
        S = x.shape[-1]
        self._f64(J, (20, g.ny, g.nx, S), "J")
        self._f64(b, (2, g.ny, g.nx, S), "b")
        self._f64(x, (2, g.ny, g.nx, S), "x")
        self._check(self._lib.henry_gs_pass(self._h, g, S, _ptr(J), _ptr(b), _ptr(x), colour, int(transpose)))
        return x

    def coarse_solve(self, J, b, g: henry_grid, solver: int = 1, precision: int = 64, transpose: bool = False):
        """x = J^{-1} b (J^{-T} b) by the coarse-grid direct solver (0 banded, 1 dense pivoted LU, 2 pivoted
        band LU)."""
        S = b.shape[-1]
        self._f64(J, (20, g.ny, g.nx, S), "J")
        self._f64(b, (2, g.ny, g.nx, S), "b")
        x = torch.empty_like(b)
        self._check(self._lib.henry_coarse_solve(self._h, solver, precision, g, S, _ptr(J), _ptr(b), _ptr(x),
                                                 int(transpose)))
        return x

    def autotune(self, theta, g: henry_grid, prob=None, opts=None):
        """Fastest solver options for this batch shape (times one Newton iteration per candidate)."""
        _check_theta(theta, self.device)
        prob = prob or problem()
        o = henry_solver_opts()
        C.memmove(C.byref(o), C.byref(opts or solver_opts()), C.sizeof(o))
        ms = C.c_double()
        self._check(self._lib.henry_autotune(self._h, C.byref(prob), C.byref(o), g, theta.shape[0], _ptr(theta),
                                             C.byref(ms)))
        return o, ms.value

    def profile(self, enable: bool):
        """Start (reset) or stop event timing of kernel classes on this context's stream."""
        self._check(self._lib.henry_profile(self._h, 1 if enable else 0))

    def profile_read(self):
        """{class: (launches, units, total_ms)} for the classes in _lib.PROF_CLASSES."""
        out = {}
        for k, name in enumerate(L.PROF_CLASSES):
            n, u, ms = C.c_longlong(), C.c_longlong(), C.c_double()
            self._check(self._lib.henry_profile_read(self._h, k, C.byref(n), C.byref(u), C.byref(ms)))
            out[name] = (n.value, u.value, ms.value)
        return out


class SaltMassQoI(torch.autograd.Function):
    """Q(theta) = salt mass in x > qoi_xmin at t = T per sample, differentiable in theta.

    forward(theta [S, 13], hx, grid, prob, opts, checkpoint_every) -> Q [S].  When theta
    needs a gradient, forward runs henry_adjoint_batch (the forward solve, then the discrete
    adjoint's reverse sweep of transposed multigrid-preconditioned solves) and keeps dQ/dtheta
    [S, 13]; otherwise it runs only the forward solve.  backward(grad_Q) returns
    grad_Q[:, None] * dQ/dtheta: the implicit-function-theorem adjoint of the converged
    implicit-Euler steps is exact for the discrete solve, so the product is the vector-Jacobian
    product of Q.  Samples that fail to converge raise HenryError (no gradient is defined).
    """

    @staticmethod
    def forward(ctx, theta, hx, g, prob, opts, checkpoint_every):
        th = theta.detach().contiguous()
        if ctx.needs_input_grad[0]:
            q, grad, st, nf = hx.adjoint(th, g, prob, opts, checkpoint_every)
            ctx.save_for_backward(grad)
        else:
            r = hx.solve(th, g, prob, opts, want_c=False)
            q, nf = r.qoi, r.nfailed
        if nf:
            raise HenryError(nf, f"{nf} samples did not converge; Q and dQ/dtheta are undefined there")
        return q

    @staticmethod
    def backward(ctx, grad_q):
        (grad,) = ctx.saved_tensors
        return grad_q[:, None] * grad, None, None, None, None, None


def salt_mass_qoi(hx: "Henry", theta, g: henry_grid, prob=None, opts=None, checkpoint_every: int = 32):
    """Q(theta) [S] through SaltMassQoI: torch.autograd.grad(Q.sum(), theta) is dQ/dtheta."""
    return SaltMassQoI.apply(theta, hx, g, prob or problem(), opts or solver_opts(), checkpoint_every)


def mlmc_run(hx: "Henry", thetas, levels, prob=None, opts=None, alpha: float = 1.0, fields: bool = True):
    """One multilevel Monte Carlo estimate (paper section 3, eq. A) in a single ragged solve.

    thetas[l]: float64 CUDA tensor [m_l, 13] for level levels[l]; level l > 0 is solved on
    its own grid and, with the same theta (coupled pair), on the next coarser grid.  All
    batches go to the library in one call, which merges batches sharing a grid and runs
    the grids concurrently.  Returns the estimator dict of Henry.mlmc_estimate plus the
    per-batch solve results.
    """
    items, idx = [], []
    for l, (th, lev) in enumerate(zip(thetas, levels)):
        items.append((th, level_grid(lev)))
        f = len(items) - 1
        c = None
        if l > 0:
            items.append((th, level_grid(levels[l - 1])))
            c = len(items) - 1
        idx.append((f, c))
    res = hx.solve_ragged(items, prob, opts, want_c=fields)
    grids = [level_grid(lev) for lev in levels]
    gf = [res[f].qoi for f, _ in idx]
    gc = [None if c is None else res[c].qoi for _, c in idx]
    cf = [res[f].c_T for f, _ in idx] if fields else None
    cc = [None if c is None else res[c].c_T for _, c in idx] if fields else None
    est = hx.mlmc_estimate(grids, gf, gc, cf, cc, alpha)
    est["results"] = res
    est["nfailed"] = sum(r.nfailed for r in res)
    return est


def mlmc_run_vc(hx: "Henry", thetas, levels, prob=None, opts=None, alpha: float = 2.0):
    """Multilevel Monte Carlo (section 3, eq. A) over the paper's own hierarchy (Table 2) with
    the vertex-centred discretisation: level l is solved on vc_level_grid(levels[l]) and, for
    l > 0, with the same theta on vc_level_grid(levels[l - 1]); all of them in one
    henry_vc_solve_batch call, concurrently.  Each level refines the mesh
    4x per direction, so alpha (the bias term's base-2 rate) defaults to 2 for a first-order
    error in h.  QoI-only: the vertex grids do not nest by 2x, so no field moments.  Returns
    the estimator dict of Henry.mlmc_estimate plus the solve results and failure count."""
    items, idx = [], []
    for l, (th, lev) in enumerate(zip(thetas, levels)):
        items.append((th, vc_level_grid(lev)))
        f = len(items) - 1
        c = None
        if l > 0:
            items.append((th, vc_level_grid(levels[l - 1])))
            c = len(items) - 1
        idx.append((f, c))
    res = hx.vc_solve_batch(items, prob, opts, want_c=False)
    grids = [vc_level_grid(lev) for lev in levels]
    gf = [res[f].qoi for f, _ in idx]
    gc = [None if c is None else res[c].qoi for _, c in idx]
    est = hx.mlmc_estimate(grids, gf, gc, None, None, alpha)
    est["results"] = res
    est["nfailed"] = sum(r.nfailed for r in res)
    return est


def mlmc_plan(Ymean_abs, V, s, eps, E0, max_level):
    """Adaptive MLMC plan from pilot statistics on levels 0..Lp (mlmc_plan in the C ABI):
    returns dict(L, m [L+1], cost, alpha, beta, gamma, c1, c2, c3, mc_cost); mc_cost is the
    cost of plain Monte Carlo at level L for the same accuracy (section 5, Test B4)."""
    n = len(V)
    m = (C.c_longlong * (max_level + 1))()
    cost = C.c_double()
    rates = (C.c_double * 7)()
    D = C.c_double * n
    L_ = L.load().mlmc_plan(n - 1, D(*Ymean_abs), D(*V), D(*s), eps, E0, max_level, m, C.byref(cost), rates)
    if L_ < 0:
        raise HenryError(L_, "invalid pilot statistics for mlmc_plan")
    return dict(L=L_, m=list(m)[:L_ + 1], cost=cost.value, alpha=rates[0], beta=rates[1], gamma=rates[2],
                c1=rates[3], c2=rates[4], c3=rates[5], mc_cost=rates[6])


def mlmc_adaptive(hx: "Henry", sampler, eps: float, prob=None, opts=None, pilot_levels: int = 3,
                  pilot_samples: int = 32, max_level: int = 5, alpha_bias: float | None = None):
    """Adaptive MLMC (section 3): pilot runs, fitted rates, level count and sample sizes, then
    the production run.

    sampler(level, n, first) -> float64 CUDA tensor [n, 13]: samples first..first+n-1 of the
    level's independent input stream (the coarse partner reuses them).  The pilot solves
    levels 0..pilot_levels (each with its coarse partner) one level at a time, so the wall
    time per sample gives s_l; the per-level mean and variance of Y_l of the QoI (salt mass
    in x > 1 at T) come from the device estimator.  mlmc_plan picks L and m_l for relative
    accuracy eps (E0 = |mean g_0| of the pilot); the production run draws fresh samples
    (first = pilot_samples) for levels 0..L in one ragged call.  The estimate's bias term uses
    the fitted alpha unless alpha_bias is given.  Raises HenryError (HENRY_EINVAL) when the
    pilot's |mean Y_l| do not decay (no positive alpha), since no level count can then be
    derived from the bias rule.
    """
    import time
    Ym, V, s = [], [], []
    for lev in range(pilot_levels + 1):
        th = sampler(lev, pilot_samples, 0)
        items = [(th, level_grid(lev))] + ([(th, level_grid(lev - 1))] if lev > 0 else [])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = hx.solve_ragged(items, prob, opts, want_c=False)
        torch.cuda.synchronize()
        s.append((time.perf_counter() - t0) / pilot_samples)
        gf = res[0].qoi.view(1, 1, -1)
        if lev == 0:
            est = hx.mlmc_estimate_series([henry_grid(1, 1, 1)], [gf], [None])
        else:
            gc = res[1].qoi.view(1, 1, -1)
            est = hx.mlmc_estimate_series([henry_grid(1, 1, 1)] * 2, [gf, gf], [None, gc])
        Ym.append(abs(float(est["Ymean"][-1, 0, 0])))
        V.append(float(est["V"][-1, 0, 0]))
    E0 = Ym[0]
    plan = mlmc_plan(Ym, V, s, eps, E0, max_level)
    Lp = plan["L"]
    thetas = [sampler(l, plan["m"][l], pilot_samples) for l in range(Lp + 1)]
    t0 = time.perf_counter()
    est = mlmc_run(hx, thetas, list(range(Lp + 1)), prob, opts,
                   alpha=plan["alpha"] if alpha_bias is None else alpha_bias, fields=False)
    torch.cuda.synchronize()
    est["wall_s"] = time.perf_counter() - t0
    est["plan"] = plan
    est["pilot"] = dict(Ymean_abs=Ym, V=V, s=s, E0=E0)
    return est


def optimal_samples(V, s, eps):
    """eq. M_ell: m_l = ceil(2 eps^-2 sqrt(V_l/s_l) sum sqrt(V_i s_i)); returns (m list, cost)."""
    n = len(V)
    m = (C.c_longlong * n)()
    cost = C.c_double()
    rc = L.load().mlmc_optimal_samples(n - 1, (C.c_double * n)(*V), (C.c_double * n)(*s), eps, m, C.byref(cost))
    if rc != 0:
        raise HenryError(rc, "invalid arguments to mlmc_optimal_samples")
    return list(m), cost.value
