"""Vertex-centred finite volumes (the paper's discretisation) -- TEST INFRASTRUCTURE ONLY.

Same balance laws, densities and boundary data as oracle.henry (paper section 2.1), on
the discretisation of section 2.3: the domain is covered with nx x ny rectangular elements
(quadrilaterals); p and c live at the (nx + 1)(ny + 1) vertices (two unknowns per vertex);
each vertex owns the box formed by the four quarter-elements around it; implicit Euler in
time; partial upwind for the convective salt flux.  The paper defers the details of the
scheme to its references, so this file states the reading it implements:

* Elements e = (i, j) span [x_i, x_i + hx] x [y_j, y_j + hy], with x_i = i hx and
  y_j = -Ly + j hy; phi and K are constant per element (the fields of oracle.henry
  evaluated at element centres).  Local vertices 0 = (i, j), 1 = (i+1, j), 2 = (i+1, j+1),
  3 = (i, j+1); bilinear shape functions N_0 = (1-s)(1-t), N_1 = s(1-t), N_2 = s t,
  N_3 = (1-s) t of the local coordinates s = (x - x_i)/hx, t = (y - y_j)/hy.
* Each element holds four box faces, the segments from its centre to its edge midpoints.
  Face k separates local vertices a_k and b_k and is crossed along +x or +y (from a to b):
      face 0: 0 -> 1, +x, at s = 1/2, t in [0, 1/2]      face 1: 1 -> 2, +y, at t = 1/2, s in [1/2, 1]
      face 2: 3 -> 2, +x, at s = 1/2, t in [1/2, 1]      face 3: 0 -> 3, +y, at t = 1/2, s in [0, 1/2]
  Fluxes are evaluated at the face midpoint (the integration point, ip): the bilinear
  gradients of p and c there, rho_ip = sum N_k rho(c_k), and Darcy
  q = -(K_e/mu)(grad p - rho_ip g) with g = (0, -g):
      F = rho_ip (q . n) |f|                                  fluid mass flux a -> b
      G = F c_conv - rho_ip phi_e D_m (grad c . n) |f|        salt mass flux a -> b
* Partial upwind: c_conv = (1 - w)(c_a + c_b)/2 + w c_up, c_up the upstream one of c_a,
  c_b, with the smallest upwind fraction that keeps the face's downstream coupling
  non-positive, w = max(0, 1 - 2 D_f / |F|), D_f = rho_ip phi_e D_m |f| / h (h = hx on
  x-faces, hy on y-faces): central (second order) where the face Peclet number
  |F| / D_f <= 2, and beyond it the convective flux upwinded just enough.
* Storage is lumped at the vertex: box_v = sum over the elements around v of
  (hx hy / 4) phi_e, R^p_v = box_v (rho(c_v) - rho(c_v^old)) / tau + sum of F out of v,
  R^c_v = box_v (rho(c_v) c_v - rho(c_v^old) c_v^old) / tau + sum of G out of v.
* Boundary data as the paper states them: on x = Lx, p = -rho1 g y and c = 1 (Dirichlet
  at those vertices); on x = 0, c = c_left (Dirichlet) and the fluid mass flux
  rho(c_left) u_in enters through each vertex's part of the side (hy, halved at the
  corners); top and bottom closed.  A Dirichlet unknown's equation is u - u_D = 0.
* Hierarchy of Table 2: level l has 16 4^l x 8 4^l elements, (16 4^l + 1)(8 4^l + 1)
  vertices and 94 4^l steps of 64 / 4^l s (T = 6016 s).

The Newton matrix is the residual's Jacobian by central differences (steps 1e-5 in c and
1e-7 rho0 g Ly in p), all vertices of one
colour (i mod 3, j mod 3) perturbed at once (a residual row depends only on the 3 x 3
vertices around it), solved by SuperLU; the Jacobian affects only the convergence of
Newton's method, not its fixed point.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .henry import Grid, Problem, SolveOptions, recharge_factor, rho, sample_fields

# face k: (a, b, axis 0 = x / 1 = y, s_ip, t_ip)
FACES = ((0, 1, 0, 0.5, 0.25), (1, 2, 1, 0.75, 0.5), (3, 2, 0, 0.5, 0.75), (0, 3, 1, 0.25, 0.5))


def level_grid(level: int) -> Grid:
    """Level l of Table 2: 16 4^l x 8 4^l elements, 94 4^l implicit-Euler steps."""
    return Grid(16 * 4 ** level, 8 * 4 ** level, 94 * 4 ** level)


def vertex_count(grid: Grid) -> int:
    return (grid.nx + 1) * (grid.ny + 1)


def shape(s, t):
    """N_0..N_3 at local (s, t)."""
    return np.array([(1 - s) * (1 - t), s * (1 - t), s * t, (1 - s) * t])


def shape_grad(s, t, hx, hy):
    """(dN/dx, dN/dy) of N_0..N_3 at local (s, t)."""
    dx = np.array([-(1 - t), 1 - t, t, -t]) / hx
    dy = np.array([-(1 - s), -s, s, 1 - s]) / hy
    return dx, dy


def upwind_fraction(F, Df):
    """w = max(0, 1 - 2 D_f/|F|), 0 where F = 0."""
    aF = np.abs(F)
    with np.errstate(divide="ignore", invalid="ignore"):
        w = np.where(aF > 0.0, 1.0 - 2.0 * Df / np.where(aF > 0.0, aF, 1.0), 0.0)
    return np.maximum(w, 0.0)


class VCDiscretisation:
    """Residual of one implicit-Euler step for one sample on the vertex grid."""

    def __init__(self, prob: Problem, grid: Grid, phi, K, u_in, tau=None):
        self.prob, self.grid = prob, grid
        self.phi, self.K = np.asarray(phi).ravel(), np.asarray(K).ravel()   # per element [j, i]
        self.u_in = u_in
        self.u_in_t = u_in
        self.hx, self.hy = grid.h(prob)
        self.tau = prob.T / grid.nsteps if tau is None else tau
        nx, ny = grid.nx, grid.ny
        self.nvx, self.nvy = nx + 1, ny + 1
        self.nv = self.nvx * self.nvy
        vid = np.arange(self.nv).reshape(self.nvy, self.nvx)
        self.vid = vid
        # element -> its four vertices (local order 0..3)
        self.ev = np.stack([vid[:-1, :-1].ravel(), vid[:-1, 1:].ravel(), vid[1:, 1:].ravel(), vid[1:, :-1].ravel()],
                           axis=1)
        self.yv = (-prob.Ly + np.arange(self.nvy) * self.hy)[:, None] * np.ones((1, self.nvx))
        self.xv = (np.arange(self.nvx) * self.hx)[None, :] * np.ones((self.nvy, 1))
        self.yv, self.xv = self.yv.ravel(), self.xv.ravel()
        self.box = np.zeros(self.nv)
        for k in range(4):
            np.add.at(self.box, self.ev[:, k], 0.25 * self.hx * self.hy * self.phi)
        self.right = vid[:, -1]
        self.left = vid[:, 0]
        self.p_dir = -prob.rho1 * prob.g * self.yv[self.right]
        # left boundary length of each left vertex
        self.left_len = np.full(self.nvy, self.hy)
        self.left_len[0] = self.left_len[-1] = 0.5 * self.hy

    def set_time(self, t):
        self.u_in_t = self.u_in * recharge_factor(self.prob, t)

    def faces(self, p, c):
        """Per element and face: F, G (a -> b), the vertices a, b, w and the upwind side."""
        pr = self.prob
        hx, hy = self.hx, self.hy
        pe, ce = p[self.ev], c[self.ev]          # [ne, 4]
        re = rho(pr, ce)
        out = []
        for a, b, axis, s, t in FACES:
            N = shape(s, t)
            dx, dy = shape_grad(s, t, hx, hy)
            dN = dx if axis == 0 else dy
            length = 0.5 * hy if axis == 0 else 0.5 * hx
            h = hx if axis == 0 else hy
            r_ip = re @ N
            gp = pe @ dN
            gc = ce @ dN
            qn = -(self.K / pr.mu) * (gp + (r_ip * pr.g if axis == 1 else 0.0))
            F = r_ip * qn * length
            Df = r_ip * self.phi * pr.Dm * length / h
            w = upwind_fraction(F, Df)
            up_a = F >= 0.0
            c_up = np.where(up_a, ce[:, a], ce[:, b])
            c_conv = (1.0 - w) * 0.5 * (ce[:, a] + ce[:, b]) + w * c_up
            G = F * c_conv - r_ip * self.phi * pr.Dm * gc * length
            out.append(dict(a=self.ev[:, a], b=self.ev[:, b], F=F, G=G, w=w, Df=Df))
        return out

    def flux_balance(self, p, c):
        """Net (fluid, salt) mass flux out of every vertex's box, boundary inflow included."""
        pr = self.prob
        Fp = np.zeros(self.nv)
        Fc = np.zeros(self.nv)
        for f in self.faces(p, c):
            np.add.at(Fp, f["a"], f["F"]); np.add.at(Fp, f["b"], -f["F"])
            np.add.at(Fc, f["a"], f["G"]); np.add.at(Fc, f["b"], -f["G"])
        qin = rho(pr, pr.c_left) * self.u_in_t * self.left_len
        Fp[self.left] -= qin
        Fc[self.left] -= qin * pr.c_left
        return Fp, Fc

    def residual(self, p, c, c_old):
        pr = self.prob
        Fp, Fc = self.flux_balance(p, c)
        Rp = self.box * (rho(pr, c) - rho(pr, c_old)) / self.tau + Fp
        Rc = self.box * (rho(pr, c) * c - rho(pr, c_old) * c_old) / self.tau + Fc
        Rp[self.right] = p[self.right] - self.p_dir
        Rc[self.right] = c[self.right] - 1.0
        Rc[self.left] = c[self.left] - pr.c_left
        return Rp, Rc

    def residual_vector(self, u, c_old):
        Rp, Rc = self.residual(u[0::2], u[1::2], c_old)
        R = np.empty(2 * self.nv)
        R[0::2], R[1::2] = Rp, Rc
        return R

    def jacobian_fd(self, p, c, c_old):
        """d(R^p, R^c)/d(p, c) by coloured central differences (unknown 2 v + {0: p, 1: c})."""
        pr = self.prob
        u = np.empty(2 * self.nv)
        u[0::2], u[1::2] = p, c
        iv, jv = np.meshgrid(np.arange(self.nvx), np.arange(self.nvy))
        colour = ((iv % 3) + 3 * (jv % 3)).ravel()
        # neighbourhood of every vertex: itself and the (up to) 8 vertices around it
        rows, cols, vals = [], [], []
        # the residual is linear in p and at most quadratic in c (apart from the upwind fraction),
        # so central differences are exact up to rounding.  In c a step of 1e-5 keeps the
        # rounding of the hydrostatic term (~rho g Ly) small against the change it measures; in
        # p a step of 1e-7 rho0 g Ly moves a face flux by ~1e-5 of itself, so it seldom carries
        # a face across the upwind fraction's kink |F| = 2 D_f.
        steps = (pr.rho0 * pr.g * pr.Ly * 1e-7, 1e-5)
        for comp in range(2):
            for col in range(9):
                vs = np.nonzero(colour == col)[0]
                if vs.size == 0:
                    continue
                e = np.zeros_like(u)
                e[2 * vs + comp] = steps[comp]
                d = (self.residual_vector(u + e, c_old) - self.residual_vector(u - e, c_old)) / (2.0 * steps[comp])
                # row r belongs to the one perturbed vertex within one cell of it
                rv = np.arange(self.nv)
                ri, rj = rv % self.nvx, rv // self.nvx
                for di in (-1, 0, 1):
                    for dj in (-1, 0, 1):
                        qi, qj = ri + di, rj + dj
                        ok = (qi >= 0) & (qi < self.nvx) & (qj >= 0) & (qj < self.nvy)
                        q = qj * self.nvx + qi
                        ok &= np.where(ok, colour[np.where(ok, q, 0)] == col, False)
                        r = rv[ok]
                        for rc in range(2):
                            rows.append(2 * r + rc)
                            cols.append(2 * q[ok] + comp)
                            vals.append(d[2 * r + rc])
        r = np.concatenate(rows); cc = np.concatenate(cols); v = np.concatenate(vals)
        keep = v != 0.0
        return sp.csc_matrix((v[keep], (r[keep], cc[keep])), shape=(2 * self.nv, 2 * self.nv))

    def boundary_outflux(self, p, c):
        """(fluid, salt) mass per unit time leaving the vertices whose fluid (salt) equation is
        a balance: the left inflow plus what the box faces carry into Dirichlet vertices."""
        pr = self.prob
        act_p = np.ones(self.nv, bool); act_p[self.right] = False
        act_c = act_p.copy(); act_c[self.left] = False
        fp = -np.sum(rho(pr, pr.c_left) * self.u_in_t * self.left_len)
        fc = 0.0
        for f in self.faces(p, c):
            a, b = f["a"], f["b"]
            fp += np.sum(f["F"][act_p[a] & ~act_p[b]]) - np.sum(f["F"][~act_p[a] & act_p[b]])
            fc += np.sum(f["G"][act_c[a] & ~act_c[b]]) - np.sum(f["G"][~act_c[a] & act_c[b]])
        return fp, fc


def initial_state(prob: Problem, grid: Grid):
    """c = 0 with the Dirichlet values c = 1 on x = Lx; p = -rho0 g y (first Newton guess),
    -rho1 g y on x = Lx."""
    nvx, nvy = grid.nx + 1, grid.ny + 1
    hx, hy = grid.h(prob)
    y = np.repeat(-prob.Ly + np.arange(nvy) * hy, nvx)
    p = -prob.rho0 * prob.g * y
    c = np.zeros(nvx * nvy)
    right = np.arange(nvy) * nvx + nvx - 1
    p[right] = -prob.rho1 * prob.g * y[right]
    c[right] = 1.0
    c[np.arange(nvy) * nvx] = prob.c_left
    return p, c


def newton_step(disc: VCDiscretisation, p, c, c_old, opts: SolveOptions):
    """One implicit-Euler step, damped as in oracle.henry.newton_step (updates scaled by
    min(1, dc_max / |dc|_inf); convergence on the unscaled update)."""
    pr = disc.prob
    p_ref = pr.rho0 * pr.g * pr.Ly
    p, c = p.copy(), c.copy()
    for it in range(1, opts.newton_maxit + 1):
        Rp, Rc = disc.residual(p, c, c_old)
        R = np.empty(2 * disc.nv); R[0::2] = Rp; R[1::2] = Rc
        d = spla.splu(disc.jacobian_fd(p, c, c_old)).solve(-R)
        dcm = np.abs(d[1::2]).max()
        lam = min(1.0, opts.dc_max / dcm) if dcm > 0.0 else 1.0
        p += lam * d[0::2]; c += lam * d[1::2]
        if max(np.abs(d[1::2]).max(), np.abs(d[0::2]).max() / p_ref) <= opts.newton_tol:
            return p, c, it, True
    return p, c, opts.newton_maxit, False


def qoi_salt_mass(prob: Problem, grid: Grid, c):
    """Salt mass sum c_v rho(c_v) |box_v n {x > qoi_xmin}| (the section-5 integrand c rho(c),
    eq. integral_s, with the vertex value constant on its box)."""
    hx, hy = grid.h(prob)
    nvx, nvy = grid.nx + 1, grid.ny + 1
    x = np.arange(nvx) * hx
    lo = np.maximum(x - 0.5 * hx, 0.0)          # the box's x-extent inside the domain
    hi = np.minimum(x + 0.5 * hx, prob.Lx)
    wx = np.maximum(0.0, hi - np.maximum(lo, prob.qoi_xmin))
    wy = np.full(nvy, hy)
    wy[0] = wy[-1] = 0.5 * hy
    cc = c.reshape(nvy, nvx)
    return float(np.sum(cc * rho(prob, cc) * wy[:, None] * wx[None, :]))


@dataclasses.dataclass
class VCResult:
    p: np.ndarray
    c: np.ndarray
    qoi: float
    newton_its: int
    converged: bool
    max_fluid_defect: float
    max_salt_defect: float
    states: list | None = None


def solve_sample(prob: Problem, grid: Grid, theta, opts: SolveOptions | None = None, keep_states=False,
                 nsteps=None, tau=None) -> VCResult:
    """Time loop for one sample on the vertex grid (Newton + sparse direct LU)."""
    opts = opts or SolveOptions()
    phi, K, u_in = sample_fields(prob, grid, theta)
    disc = VCDiscretisation(prob, grid, phi, K, u_in, tau=tau)
    p, c = initial_state(prob, grid)
    its, ok = 0, True
    dmax_f = dmax_s = 0.0
    act_p = np.ones(disc.nv, bool); act_p[disc.right] = False
    act_c = act_p.copy(); act_c[disc.left] = False
    states = [(p.copy(), c.copy())] if keep_states else None
    for n in range(nsteps if nsteps is not None else grid.nsteps):
        c_old = c.copy()
        disc.set_time((n + 1) * disc.tau)
        p, c, k, conv = newton_step(disc, p, c, c_old, opts)
        its += k
        ok = ok and conv
        ff, fs = disc.boundary_outflux(p, c)
        st_f = np.sum((disc.box * (rho(prob, c) - rho(prob, c_old)))[act_p])
        st_s = np.sum((disc.box * (rho(prob, c) * c - rho(prob, c_old) * c_old))[act_c])
        scale = disc.tau * prob.rho0 * u_in * prob.Ly
        dmax_f = max(dmax_f, abs(st_f + disc.tau * ff) / scale)
        dmax_s = max(dmax_s, abs(st_s + disc.tau * fs) / scale)
        if keep_states:
            states.append((p.copy(), c.copy()))
    return VCResult(p, c, qoi_salt_mass(prob, grid, c), its, ok, dmax_f, dmax_s, states)
