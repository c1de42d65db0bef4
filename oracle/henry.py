"""Plain FP64 oracle of the per-realisation Henry solve -- TEST INFRASTRUCTURE ONLY.

Model (paper section 2.1): fluid mass balance d_t(phi rho) + div(rho q) = 0 and
salt mass balance d_t(phi rho c) + div(rho c q - rho phi D grad c) = 0 with Darcy
q = -(K/mu)(grad p - rho g), g = (0, -g), linear density rho(c) = rho0 + (rho1-rho0) c,
constant viscosity, dispersion D = phi D_m I, isotropic K, no Boussinesq
approximation.  c(0) = 0.  Right side: hydrostatic seawater pressure
p = -rho1 g y; left side: fresh-water inflow at c = c_left; top and bottom closed.

Discretisation (a cell-centred reading of section 2.3; implicit Euler in time):
cells (i, j) of size hx x hy, centres x_i = (i+1/2) hx, y_j = -Ly + (j+1/2) hy.
For an interior face f between P and its east/north neighbour Q:
  K_f = 2 K_P K_Q / (K_P + K_Q)      rho_f = (rho(c_P) + rho(c_Q)) / 2
  phi_f = (phi_P + phi_Q) / 2
  u_f = -(K_f/mu) [ (p_Q - p_P)/d + rho_f g n_y ]      (n_y = 1 on north faces)
  F_f = rho_f u_f A_f                                    (fluid mass flux, P -> Q)
  G_f = F_f c_up - rho_f phi_f D_m (c_Q - c_P) A_f / d    (c_up = c_P if F_f >= 0)
with d the centre distance and A_f the face length.  Residuals per cell:
  R^p_P = V phi_P (rho(c_P) - rho(c_P^old)) / tau + sum_f F_f,out
  R^c_P = V phi_P (rho(c_P) c_P - rho(c_P^old) c_P^old) / tau + sum_f G_f,out
Left face: F_out = -rho(c_left) u_in hy, G_out = F_out c_left + 2 rho(c_P) phi_P D_m (c_P - c_left) hy/hx.
Right face: p_b = -rho1 g y_j, u = -(K_P/mu)(p_b - p_P)/(hx/2); inflow (u < 0) carries
rho1 and c = 1, outflow carries rho(c_P) and c_P; in the Dirichlet variant (paper's
c = 1 on the whole right side) a diffusive term 2 rho(c_P) phi_P D_m (c_P - 1) hy/hx is added.

Each Newton system is solved by SuperLU (scipy.sparse.linalg.splu): no Krylov or
multigrid, so the result is the fixed point of the discrete equations.
"""
from __future__ import annotations

import dataclasses
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .kl import KL2D


@dataclasses.dataclass
class Problem:
    """Physical constants (paper Table 1, with g and rho1 of the studied workload)."""
    Lx: float = 2.0
    Ly: float = 1.0
    T: float = 36000.0
    rho0: float = 1000.0
    rho1: float = 1025.0
    mu: float = 1e-3
    g: float = 9.81
    Dm: float = 1.88571e-5
    phi_mean: float = 0.35
    phi_amp: float = 0.2
    phi_min: float = 0.2
    phi_max: float = 0.5
    K_mean: float = 1.020408e-9
    logK_amp: float = 0.5
    corr_len: float = 0.5
    q_in: float = 6.6e-5
    q_in_amp: float = 0.1
    n_kl_phi: int = 4
    n_kl_logK: int = 8
    right_c_dirichlet: bool = False
    c_left: float = 0.0
    field_model: str = "kl"         # "kl": KL fields above; "paper": section 4 porosity and K
    kappa_kc: float = 2.088415e-8   # Kozeny-Carman scale kappa_KC (Table 1), m^2
    recharge_omega: float = 0.0     # left inflow u_in (1 + sin(omega t)); 0: constant in time
    qoi_xmin: float = 1.0           # QoI region: cells whose centre lies in x > qoi_xmin


def paper_problem(**kw) -> Problem:
    """The paper's own stochastic model (section 4).

    Porosity eq. poro_2levels (xi_1 = theta[0], xi_2 = theta[1]), permeability by
    Kozeny-Carman (eq. e_perm_Kozeny_Carman), recharge eq. e_recharge_of_param:
    6.6e-2 (1 + 0.5 xi_3)(1 + sin(pi t / 40)) kg/s over the 1 m left face, i.e. the
    inflow velocity 6.6e-5 (1 + 0.5 xi_3)(1 + sin(pi t / 40)) m/s (xi_3 = theta[12]),
    and the horizon T = 6016 s of section 4.
    """
    d = dict(field_model="paper", q_in_amp=0.5, recharge_omega=np.pi / 40.0, T=6016.0)
    d.update(kw)
    return Problem(**d)


@dataclasses.dataclass
class Grid:
    nx: int
    ny: int
    nsteps: int

    def h(self, prob: Problem):
        return prob.Lx / self.nx, prob.Ly / self.ny


def cell_centres(prob: Problem, grid: Grid):
    hx, hy = grid.h(prob)
    x = (np.arange(grid.nx) + 0.5) * hx
    y = -prob.Ly + (np.arange(grid.ny) + 0.5) * hy
    X, Y = np.meshgrid(x, y)   # [ny, nx]
    return X, Y


_KL_CACHE = {}


def kl_basis(prob: Problem) -> KL2D:
    key = (prob.Lx, prob.Ly, prob.corr_len, max(prob.n_kl_phi, prob.n_kl_logK))
    if key not in _KL_CACHE:
        _KL_CACHE[key] = KL2D(prob.Lx, prob.Ly, prob.corr_len, key[3])
    return _KL_CACHE[key]


def paper_porosity(X, Y, xi1, xi2, phi_hat=0.35):
    """Section 4, eq. poro_2levels: phi = phi_hat C0 C1 C2 with
    C0 = 1.2 (1 + 0.2 xi_1) below y = -0.8 and 1 above (a second layer),
    C1 = 1 + 0.15 (xi_2 cos(pi x/2) - xi_2 sin(2 pi y) + xi_1 cos(2 pi x)) (large scales),
    C2 = 1 + 0.2 (xi_1 sin(64 pi x) + xi_2 sin(32 pi y)) (small scales)."""
    C0 = np.where(Y < -0.8, 1.2 * (1.0 + 0.2 * xi1), 1.0)
    C1 = 1.0 + 0.15 * (xi2 * np.cos(np.pi * X / 2.0) - xi2 * np.sin(2.0 * np.pi * Y) + xi1 * np.cos(2.0 * np.pi * X))
    C2 = 1.0 + 0.2 * (xi1 * np.sin(64.0 * np.pi * X) + xi2 * np.sin(32.0 * np.pi * Y))
    return phi_hat * C0 * C1 * C2


def kozeny_carman(prob: Problem, phi):
    """eq. e_perm_Kozeny_Carman: K = kappa_KC phi^3 / (1 - phi^2)."""
    return prob.kappa_kc * phi ** 3 / (1.0 - phi ** 2)


def recharge_factor(prob: Problem, t):
    """Time factor of the left inflow, 1 + sin(omega t) (eq. e_recharge_of_param with
    omega = pi/40); exactly 1 for the constant-inflow model (omega = 0)."""
    return 1.0 + np.sin(prob.recharge_omega * t)


def sample_fields(prob: Problem, grid: Grid, theta):
    """phi[ny,nx], K[ny,nx], u_in for one theta[13], evaluated at cell centres.

    KL model:
      phi = clip(phi_mean (1 + phi_amp sum_{k<4} sqrt(lam_k) xi_k e_k), phi_min, phi_max)
      ln K = ln K_mean + logK_amp sum_{k<8} sqrt(lam_k) eta_k e_k
    paper model: phi by eq. poro_2levels, K = kappa_KC phi^3 / (1 - phi^2).
    Both: u_in = q_in (1 + q_in_amp zeta) (times the recharge time factor per step).
    """
    theta = np.asarray(theta, dtype=np.float64)
    X, Y = cell_centres(prob, grid)
    if prob.field_model == "paper":
        phi = paper_porosity(X, Y, theta[0], theta[1], prob.phi_mean)
        return phi, kozeny_carman(prob, phi), prob.q_in * (1.0 + prob.q_in_amp * theta[12])
    if prob.field_model != "kl":
        raise ValueError(prob.field_model)
    kl = kl_basis(prob)
    E = kl.table(X, Y)
    sl = np.sqrt(kl.lam)
    s_phi = np.zeros_like(X)
    for k in range(prob.n_kl_phi):
        s_phi += sl[k] * theta[k] * E[k]
    phi_raw = prob.phi_mean * (1.0 + prob.phi_amp * s_phi)
    phi = np.clip(phi_raw, prob.phi_min, prob.phi_max)
    s_k = np.zeros_like(X)
    for k in range(prob.n_kl_logK):
        s_k += sl[k] * theta[4 + k] * E[k]
    K = np.exp(np.log(prob.K_mean) + prob.logK_amp * s_k)
    u_in = prob.q_in * (1.0 + prob.q_in_amp * theta[12])
    return phi, K, u_in


def rho(prob: Problem, c):
    return prob.rho0 + (prob.rho1 - prob.rho0) * c


class Discretisation:
    """Residual and analytic Jacobian of one implicit-Euler step for one sample."""

    def __init__(self, prob: Problem, grid: Grid, phi, K, u_in, tau=None):
        self.prob, self.grid = prob, grid
        self.phi, self.K, self.u_in = phi, K, u_in
        self.u_in_t = u_in          # inflow at the time level being solved for
        self.hx, self.hy = grid.h(prob)
        self.tau = prob.T / grid.nsteps if tau is None else tau
        X, Y = cell_centres(prob, grid)
        self.yc = Y
        ny, nx = grid.ny, grid.nx
        self.nc = nx * ny
        idx = np.arange(self.nc).reshape(ny, nx)
        self.idx = idx
        # face lists: P -> Q (east, then north)
        self.eP, self.eQ = idx[:, :-1].ravel(), idx[:, 1:].ravel()
        self.nP, self.nQ = idx[:-1, :].ravel(), idx[1:, :].ravel()

    def set_time(self, t):
        """Boundary data of the implicit-Euler step that ends at time t."""
        self.u_in_t = self.u_in * recharge_factor(self.prob, t)

    # -- fluxes -------------------------------------------------------------
    def _face(self, p, c, P, Q, north):
        pr = self.prob
        hx, hy = self.hx, self.hy
        phi, K = self.phi.ravel(), self.K.ravel()
        d, A = (hy, hx) if north else (hx, hy)
        Kf = 2.0 * K[P] * K[Q] / (K[P] + K[Q])
        rf = 0.5 * (rho(pr, c[P]) + rho(pr, c[Q]))
        phif = 0.5 * (phi[P] + phi[Q])
        grav = rf * pr.g if north else 0.0
        u = -(Kf / pr.mu) * ((p[Q] - p[P]) / d + grav)
        F = rf * u * A
        up = F >= 0.0
        cup = np.where(up, c[P], c[Q])
        Gd = rf * phif * pr.Dm * (c[Q] - c[P]) * A / d
        G = F * cup - Gd
        return dict(Kf=Kf, rf=rf, phif=phif, u=u, F=F, up=up, cup=cup, G=G, d=d, A=A)

    def _right(self, p, c):
        pr = self.prob
        hx, hy = self.hx, self.hy
        P = self.idx[:, -1]
        pb = -pr.rho1 * pr.g * self.yc[:, -1]
        KP = self.K.ravel()[P]
        u = -(KP / pr.mu) * (pb - p[P]) / (0.5 * hx)
        inflow = u < 0.0
        rb = np.where(inflow, pr.rho1, rho(pr, c[P]))
        F = rb * u * hy
        G = F * np.where(inflow, 1.0, c[P])
        if pr.right_c_dirichlet:
            G = G + 2.0 * rho(pr, c[P]) * self.phi.ravel()[P] * pr.Dm * (c[P] - 1.0) * hy / hx
        return P, u, inflow, F, G

    def _left(self, p, c):
        pr = self.prob
        hx, hy = self.hx, self.hy
        P = self.idx[:, 0]
        F = -rho(pr, pr.c_left) * self.u_in_t * hy * np.ones(len(P))
        G = F * pr.c_left + 2.0 * rho(pr, c[P]) * self.phi.ravel()[P] * pr.Dm * (c[P] - pr.c_left) * hy / hx
        return P, F, G

    def residual(self, p, c, c_old):
        """R^p, R^c (flat arrays over cells, row-major [j, i])."""
        pr = self.prob
        phi = self.phi.ravel()
        V = self.hx * self.hy
        Rp = V * phi * (rho(pr, c) - rho(pr, c_old)) / self.tau
        Rc = V * phi * (rho(pr, c) * c - rho(pr, c_old) * c_old) / self.tau
        for P, Q, north in ((self.eP, self.eQ, False), (self.nP, self.nQ, True)):
            f = self._face(p, c, P, Q, north)
            np.add.at(Rp, P, f["F"]); np.add.at(Rp, Q, -f["F"])
            np.add.at(Rc, P, f["G"]); np.add.at(Rc, Q, -f["G"])
        P, F, G = self._left(p, c)
        Rp[P] += F; Rc[P] += G
        P, _, _, F, G = self._right(p, c)
        Rp[P] += F; Rc[P] += G
        return Rp, Rc

    def boundary_outflux(self, p, c):
        """(fluid, salt) mass leaving through the boundary per unit time."""
        _, F1, G1 = self._left(p, c)
        _, _, _, F2, G2 = self._right(p, c)
        return F1.sum() + F2.sum(), G1.sum() + G2.sum()

    def jacobian(self, p, c):
        """Analytic d(R^p, R^c)/d(p, c) as CSC; unknown 2*cell + {0: p, 1: c}.

        The upwind selections are taken from the current state and held fixed.
        """
        pr = self.prob
        dr = pr.rho1 - pr.rho0
        phi = self.phi.ravel()
        V = self.hx * self.hy
        rows, cols, vals = [], [], []

        def add(r, cc, v):
            rows.append(np.asarray(r)); cols.append(np.asarray(cc)); vals.append(np.asarray(v, dtype=np.float64))

        n = self.nc
        allc = np.arange(n)
        # storage
        add(2 * allc, 2 * allc + 1, V * phi * dr / self.tau)
        add(2 * allc + 1, 2 * allc + 1, V * phi * (pr.rho0 + 2.0 * dr * c) / self.tau)
        for P, Q, north in ((self.eP, self.eQ, False), (self.nP, self.nQ, True)):
            f = self._face(p, c, P, Q, north)
            a = f["rf"] * (f["Kf"] / pr.mu) * f["A"] / f["d"]            # dF/dp_P = -dF/dp_Q
            dudc = -(f["Kf"] / pr.mu) * pr.g * 0.5 * dr if north else 0.0
            bF = 0.5 * dr * f["u"] * f["A"] + f["rf"] * f["A"] * dudc      # dF/dc_P = dF/dc_Q
            w = f["A"] / f["d"]
            dc = c[Q] - c[P]
            dGd_dcP = 0.5 * dr * f["phif"] * pr.Dm * dc * w - f["rf"] * f["phif"] * pr.Dm * w
            dGd_dcQ = 0.5 * dr * f["phif"] * pr.Dm * dc * w + f["rf"] * f["phif"] * pr.Dm * w
            cup, F, up = f["cup"], f["F"], f["up"]
            dG_dcP = bF * cup + np.where(up, F, 0.0) - dGd_dcP
            dG_dcQ = bF * cup + np.where(up, 0.0, F) - dGd_dcQ
            for sgn, R in ((1.0, P), (-1.0, Q)):
                add(2 * R, 2 * P, sgn * a)
                add(2 * R, 2 * Q, -sgn * a)
                add(2 * R, 2 * P + 1, sgn * bF)
                add(2 * R, 2 * Q + 1, sgn * bF)
                add(2 * R + 1, 2 * P, sgn * a * cup)
                add(2 * R + 1, 2 * Q, -sgn * a * cup)
                add(2 * R + 1, 2 * P + 1, sgn * dG_dcP)
                add(2 * R + 1, 2 * Q + 1, sgn * dG_dcQ)
        # left boundary (flux fixed; only the diffusive salt term depends on c_P)
        P = self.idx[:, 0]
        w = self.hy / self.hx
        add(2 * P + 1, 2 * P + 1, 2.0 * phi[P] * pr.Dm * w * (dr * (c[P] - pr.c_left) + rho(pr, c[P])))
        # right boundary
        P, u, inflow, F, G = self._right(p, c)
        KP = self.K.ravel()[P]
        dudp = 2.0 * KP / (pr.mu * self.hx)
        rb = np.where(inflow, pr.rho1, rho(pr, c[P]))
        dFdp = rb * self.hy * dudp
        dFdc = np.where(inflow, 0.0, dr * u * self.hy)
        cb = np.where(inflow, 1.0, c[P])
        add(2 * P, 2 * P, dFdp)
        add(2 * P, 2 * P + 1, dFdc)
        add(2 * P + 1, 2 * P, cb * dFdp)
        add(2 * P + 1, 2 * P + 1, cb * dFdc + np.where(inflow, 0.0, F))
        if pr.right_c_dirichlet:
            add(2 * P + 1, 2 * P + 1, 2.0 * phi[P] * pr.Dm * w * (dr * (c[P] - 1.0) + rho(pr, c[P])))
        r = np.concatenate(rows); cc = np.concatenate(cols); v = np.concatenate(vals)
        return sp.csc_matrix((v, (r, cc)), shape=(2 * n, 2 * n))


def initial_state(prob: Problem, grid: Grid):
    """c^0 = 0 (paper section 2.1); p^0 = -rho0 g y is only the first Newton guess."""
    X, Y = cell_centres(prob, grid)
    return (-prob.rho0 * prob.g * Y).ravel(), np.zeros(grid.nx * grid.ny)


@dataclasses.dataclass
class SolveOptions:
    newton_tol: float = 1e-9      # |dc|_inf <= tol and |dp|_inf <= tol * rho0 g Ly
    newton_maxit: int = 100
    dc_max: float = 1.0           # per-iteration limit on |dc|_inf (update scaled down)
    stagnate: bool = False        # iterate until the update stops shrinking (FD checks)


def newton_step(disc: Discretisation, p, c, c_old, opts: SolveOptions):
    """One implicit-Euler step; returns (p, c, iterations, converged).

    Newton's method (paper section 2.3) from the previous state.  The paper
    reports two iterations per step at its step size; with 750 s steps the
    first step (inconsistent initial pressure, strong density-driven inflow)
    needs globalisation, so each update is scaled by min(1, dc_max/|dc|_inf).
    The scaling does not move the fixed point.  Convergence is declared on
    the size of the (unscaled) update.
    """
    pr = disc.prob
    p_ref = pr.rho0 * pr.g * pr.Ly
    p, c = p.copy(), c.copy()
    prev = np.inf
    for it in range(1, opts.newton_maxit + 1):
        Rp, Rc = disc.residual(p, c, c_old)
        R = np.empty(2 * disc.nc); R[0::2] = Rp; R[1::2] = Rc
        J = disc.jacobian(p, c)
        d = spla.splu(J).solve(-R)
        dcm = np.abs(d[1::2]).max()
        lam = min(1.0, opts.dc_max / dcm) if dcm > 0.0 else 1.0
        p += lam * d[0::2]; c += lam * d[1::2]
        size = max(np.abs(d[1::2]).max(), np.abs(d[0::2]).max() / p_ref)
        if opts.stagnate:
            # only once the quadratic phase is reached: stop when the update stops shrinking
            if size < 1e-15 or (size < 1e-8 and size >= 0.5 * prev):
                return p, c, it, True
            prev = size
        elif size <= opts.newton_tol:
            return p, c, it, True
    return p, c, opts.newton_maxit, False


def qoi_salt_mass(prob: Problem, grid: Grid, c):
    """Salt mass in x > qoi_xmin = 1 m (the paper's Q_S integrand c rho(c) of section 5,
    eq. integral_s, over the cells whose centre lies in that part of the domain)."""
    X, _ = cell_centres(prob, grid)
    hx, hy = grid.h(prob)
    cc = c.reshape(grid.ny, grid.nx)
    m = X > prob.qoi_xmin
    return float(np.sum((cc * rho(prob, cc))[m]) * hx * hy)


# Time-resolved QoIs of section 5: Q_S (eq. integral_s), Q_FW (eq. integral_fw) and the
# box integrals Q_1..Q_15 (eq. integral_box) around the points of eq. 12points.
FW_THRESHOLD = 0.012178
BOX_POINTS = [(x, y) for y in (-0.95, -0.75, -0.50) for x in (0.90, 1.15, 1.40, 1.65, 1.90)]
BOX_HALF = 0.1
N_SERIES = 2 + len(BOX_POINTS)


def _interval_overlap(a0, a1, b0, b1):
    """Length of [a0, a1] intersected with [b0, b1] (0 when disjoint)."""
    return np.maximum(0.0, np.minimum(a1, b1) - np.maximum(a0, b0))


def series_qois(prob: Problem, grid: Grid, c):
    """[Q_S, Q_FW, Q_1, ..., Q_15] of one state c (flat, row-major [j, i]).

    The cell-wise constant concentration is integrated exactly: Q_S = sum c rho(c) |cell|,
    Q_FW = sum over cells with c <= 0.012178 of |cell|, Q_i = sum c rho(c) |cell n Delta_i|
    with Delta_i = [x_i - 0.1, x_i + 0.1] x [y_i - 0.1, y_i + 0.1] (parts outside the
    domain contribute nothing).
    """
    hx, hy = grid.h(prob)
    cc = c.reshape(grid.ny, grid.nx)
    m = cc * rho(prob, cc)
    out = np.empty(N_SERIES)
    out[0] = m.sum() * hx * hy
    out[1] = np.count_nonzero(cc <= FW_THRESHOLD) * hx * hy
    xe = np.arange(grid.nx + 1) * hx                 # cell edges
    ye = -prob.Ly + np.arange(grid.ny + 1) * hy
    for b, (bx, by) in enumerate(BOX_POINTS):
        wx = _interval_overlap(xe[:-1], xe[1:], bx - BOX_HALF, bx + BOX_HALF)   # [nx]
        wy = _interval_overlap(ye[:-1], ye[1:], by - BOX_HALF, by + BOX_HALF)   # [ny]
        out[2 + b] = float(wy @ m @ wx)
    return out


@dataclasses.dataclass
class SampleResult:
    p: np.ndarray
    c: np.ndarray
    qoi: float
    newton_its: int
    converged: bool
    max_fluid_defect: float
    max_salt_defect: float
    c_min: float
    c_max: float
    states: list | None = None
    series: np.ndarray | None = None    # [nsteps, N_SERIES] after every step (series=True)


def solve_sample(prob: Problem, grid: Grid, theta, opts: SolveOptions | None = None,
                 keep_states=False, nsteps=None, series=False, start=None) -> SampleResult:
    """Time loop for one sample (plain Newton + sparse direct LU).

    Runs steps n0 .. n0 + nsteps - 1 (all steps by default) from the state (p, c) after
    step n0; start = (n0, p, c), or None for the initial state (n0 = 0).
    """
    opts = opts or SolveOptions()
    phi, K, u_in = sample_fields(prob, grid, theta)
    disc = Discretisation(prob, grid, phi, K, u_in)
    if start is None:
        n0 = 0
        p, c = initial_state(prob, grid)
    else:
        n0 = int(start[0])
        p, c = np.array(start[1], dtype=np.float64), np.array(start[2], dtype=np.float64)
    V = disc.hx * disc.hy
    phif = phi.ravel()
    its, ok = 0, True
    dmax_f = dmax_s = 0.0
    cmin, cmax = 0.0, 0.0
    states = [(p.copy(), c.copy())] if keep_states else None
    ser = [] if series else None
    for n in range(n0, n0 + (nsteps if nsteps is not None else grid.nsteps - n0)):
        c_old = c.copy()
        disc.set_time((n + 1) * disc.tau)    # implicit Euler: boundary data at the new time
        p, c, k, conv = newton_step(disc, p, c, c_old, opts)
        its += k
        ok = ok and conv
        # global balance: storage change + tau * boundary outflux = 0 (interior fluxes cancel)
        ff, fs = disc.boundary_outflux(p, c)
        st_f = np.sum(V * phif * (rho(prob, c) - rho(prob, c_old)))
        st_s = np.sum(V * phif * (rho(prob, c) * c - rho(prob, c_old) * c_old))
        scale = disc.tau * prob.rho0 * u_in * prob.Ly
        dmax_f = max(dmax_f, abs(st_f + disc.tau * ff) / scale)
        dmax_s = max(dmax_s, abs(st_s + disc.tau * fs) / scale)
        cmin, cmax = min(cmin, c.min()), max(cmax, c.max())
        if keep_states:
            states.append((p.copy(), c.copy()))
        if series:
            ser.append(series_qois(prob, grid, c))
    return SampleResult(p, c, qoi_salt_mass(prob, grid, c), its, ok, dmax_f, dmax_s, cmin, cmax, states,
                        np.array(ser) if series else None)


def _solve_one(args):
    prob, grid, th, opts, series = args
    r = solve_sample(prob, grid, th, opts, series=series)
    r.states = None
    return r


def solve_batch(prob: Problem, grid: Grid, theta, opts: SolveOptions | None = None, processes: int = 1,
                series: bool = False):
    """Solve every sample of theta[S, 13]; optional process pool (samples are independent)."""
    theta = np.asarray(theta)
    jobs = [(prob, grid, theta[s], opts, series) for s in range(theta.shape[0])]
    if processes <= 1:
        return [_solve_one(j) for j in jobs]
    import multiprocessing as mp
    with mp.get_context("fork").Pool(processes) as pool:
        return pool.map(_solve_one, jobs)
