"""Discrete adjoint of the implicit-Euler / Newton solve -- TEST INFRASTRUCTURE ONLY.

Each converged step n satisfies R^n(u^n, u^{n-1}; theta) = 0, and the QoI is
Q(u^r).  With the Lagrangian Q + sum_n lam_n^T R^n, stationarity in u^n gives
(implicit-function-theorem adjoint of the converged steps, not of unrolled Newton):
  J_r^T lam_r = -dQ/du^r
  J_n^T lam_n = -(dR^{n+1}/du^n)^T lam_{n+1},   n = r-1 .. 1
  dQ/dtheta   = sum_n lam_n^T dR^n/dtheta
with J_n = dR^n/du^n at u^n.  R^{n+1} depends on u^n only through the storage
terms in c^n (diagonal).  u^0 does not depend on theta (c^0 = 0, p^0 is a guess).
Every transposed system is solved with SuperLU (trans='T').
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from . import henry as H


def param_sensitivity_T(disc: H.Discretisation, p, c, c_old, lp, lc):
    """Contract lam^T dR/d(phi, K, u_in) for one step.

    Returns (g_phi[cells], g_K[cells], g_uin) with g_phi_P = sum lam * dR/dphi_P, etc.
    """
    pr = disc.prob
    phi = disc.phi.ravel()
    K = disc.K.ravel()
    V = disc.hx * disc.hy
    n = disc.nc
    g_phi = np.zeros(n)
    g_K = np.zeros(n)
    # storage terms
    g_phi += lp * V * (H.rho(pr, c) - H.rho(pr, c_old)) / disc.tau
    g_phi += lc * V * (H.rho(pr, c) * c - H.rho(pr, c_old) * c_old) / disc.tau
    for P, Q, north in ((disc.eP, disc.eQ, False), (disc.nP, disc.nQ, True)):
        f = disc._face(p, c, P, Q, north)
        w = f["A"] / f["d"]
        # G = F c_up - rho_f phi_f Dm (c_Q - c_P) w, phi_f = (phi_P + phi_Q)/2
        dG_dphi = -0.5 * f["rf"] * pr.Dm * (c[Q] - c[P]) * w       # same for P and Q
        lam_diff_c = lc[P] - lc[Q]                                 # row P gets +, row Q gets -
        np.add.at(g_phi, P, lam_diff_c * dG_dphi)
        np.add.at(g_phi, Q, lam_diff_c * dG_dphi)
        # K_f = 2 K_P K_Q / (K_P + K_Q); F and the advective part of G are linear in K_f
        s = K[P] + K[Q]
        dKf_dKP = 2.0 * K[Q] ** 2 / s ** 2
        dKf_dKQ = 2.0 * K[P] ** 2 / s ** 2
        dF_dKf = f["F"] / f["Kf"]
        dG_dKf = f["cup"] * dF_dKf
        t = (lp[P] - lp[Q]) * dF_dKf + (lc[P] - lc[Q]) * dG_dKf
        np.add.at(g_K, P, t * dKf_dKP)
        np.add.at(g_K, Q, t * dKf_dKQ)
    w = disc.hy / disc.hx
    # left face: diffusive salt term depends on phi_P; fluid flux on u_in
    P = disc.idx[:, 0]
    g_phi[P] += lc[P] * 2.0 * H.rho(pr, c[P]) * pr.Dm * (c[P] - pr.c_left) * w
    dF_duin = -H.rho(pr, pr.c_left) * disc.hy
    g_uin = float(np.sum(lp[P] * dF_duin + lc[P] * dF_duin * pr.c_left))
    # right face: flux linear in K_P
    P, u, inflow, F, G = disc._right(p, c)
    Gadv = F * np.where(inflow, 1.0, c[P])
    g_K[P] += (lp[P] * F + lc[P] * Gadv) / K[P]
    if pr.right_c_dirichlet:
        g_phi[P] += lc[P] * 2.0 * H.rho(pr, c[P]) * pr.Dm * (c[P] - 1.0) * w
    return g_phi, g_K, g_uin


def qoi_gradient_state(prob, grid, c):
    """dQ/dc for Q = sum_{x > 1} c rho(c) V."""
    X, _ = H.cell_centres(prob, grid)
    hx, hy = grid.h(prob)
    dr = prob.rho1 - prob.rho0
    m = (X > prob.qoi_xmin).ravel()
    return np.where(m, (prob.rho0 + 2.0 * dr * c) * hx * hy, 0.0)


def theta_jacobians(prob, grid, theta):
    """dphi/dtheta [13, cells], dK/dtheta [13, cells], du_in/dzeta (the base inflow).

    KL model: phi depends on xi_1..4 (zero where clipped), K on eta_1..8 through ln K.
    Paper model (section 4): phi = phi_hat C0 C1 C2 of eq. poro_2levels depends on xi_1 =
    theta[0] and xi_2 = theta[1] through the product rule, and K = kappa phi^3 / (1 - phi^2)
    (eq. e_perm_Kozeny_Carman) through phi: dK/dphi = kappa phi^2 (3 - phi^2) / (1 - phi^2)^2.
    """
    duin = prob.q_in * prob.q_in_amp
    if prob.field_model == "paper":
        X, Y = H.cell_centres(prob, grid)
        xi1, xi2 = float(theta[0]), float(theta[1])
        low = Y < -0.8
        C0 = np.where(low, 1.2 * (1.0 + 0.2 * xi1), 1.0)
        C1 = 1.0 + 0.15 * (xi2 * np.cos(np.pi * X / 2.0) - xi2 * np.sin(2.0 * np.pi * Y) + xi1 * np.cos(2.0 * np.pi * X))
        C2 = 1.0 + 0.2 * (xi1 * np.sin(64.0 * np.pi * X) + xi2 * np.sin(32.0 * np.pi * Y))
        dC0_1 = np.where(low, 1.2 * 0.2, 0.0)
        dC1_1 = 0.15 * np.cos(2.0 * np.pi * X)
        dC2_1 = 0.2 * np.sin(64.0 * np.pi * X)
        dC1_2 = 0.15 * (np.cos(np.pi * X / 2.0) - np.sin(2.0 * np.pi * Y))
        dC2_2 = 0.2 * np.sin(32.0 * np.pi * Y)
        ph = prob.phi_mean
        dphi = np.zeros((13, X.size))
        dphi[0] = (ph * (dC0_1 * C1 * C2 + C0 * dC1_1 * C2 + C0 * C1 * dC2_1)).ravel()
        dphi[1] = (ph * (C0 * dC1_2 * C2 + C0 * C1 * dC2_2)).ravel()
        phi = (ph * C0 * C1 * C2).ravel()
        dKdphi = prob.kappa_kc * phi ** 2 * (3.0 - phi ** 2) / (1.0 - phi ** 2) ** 2
        return dphi, dphi * dKdphi, duin
    kl = H.kl_basis(prob)
    X, Y = H.cell_centres(prob, grid)
    E = kl.table(X, Y).reshape(len(kl.lam), -1)
    sl = np.sqrt(kl.lam)
    theta = np.asarray(theta, dtype=np.float64)
    s_phi = sum(sl[k] * theta[k] * E[k] for k in range(prob.n_kl_phi))
    raw = prob.phi_mean * (1.0 + prob.phi_amp * s_phi)
    inside = (raw > prob.phi_min) & (raw < prob.phi_max)
    dphi = np.zeros((13, X.size))
    for k in range(prob.n_kl_phi):
        dphi[k] = np.where(inside, prob.phi_mean * prob.phi_amp * sl[k] * E[k], 0.0)
    _, K, _ = H.sample_fields(prob, grid, theta)
    Kf = K.ravel()
    dK = np.zeros((13, X.size))
    for k in range(prob.n_kl_logK):
        dK[4 + k] = prob.logK_amp * sl[k] * E[k] * Kf
    return dphi, dK, duin


def adjoint_gradient(prob, grid, theta, opts: H.SolveOptions | None = None):
    """(Q, dQ/dtheta[13]) for one sample via the reverse sweep over stored states.

    Under a periodic recharge the inflow of step k is u_in (1 + sin(omega t_k)) at the end
    of the step, t_k = k tau, so step k's sensitivity to the base inflow carries that factor.
    """
    opts = opts or H.SolveOptions(stagnate=True)
    res = H.solve_sample(prob, grid, theta, opts, keep_states=True)
    phi, K, u_in = H.sample_fields(prob, grid, theta)
    disc = H.Discretisation(prob, grid, phi, K, u_in)
    st = res.states
    r = len(st) - 1
    n = disc.nc
    dr = prob.rho1 - prob.rho0
    V = disc.hx * disc.hy
    phif = phi.ravel()
    g_phi = np.zeros(n)
    g_K = np.zeros(n)
    g_uin = 0.0
    rhs = np.zeros(2 * n)
    rhs[1::2] = -qoi_gradient_state(prob, grid, st[r][1])
    for k in range(r, 0, -1):
        p, c = st[k]
        c_old = st[k - 1][1]
        J = disc.jacobian(p, c)
        lam = spla.splu(J).solve(rhs, trans="T")
        lp, lc = lam[0::2], lam[1::2]
        a, b, u = param_sensitivity_T(disc, p, c, c_old, lp, lc)
        g_phi += a; g_K += b; g_uin += u * H.recharge_factor(prob, k * disc.tau)
        # -(dR^k / dc^{k-1})^T lam_k  (storage terms only)
        rhs = np.zeros(2 * n)
        rhs[1::2] = lp * V * phif * dr / disc.tau + lc * V * phif * (prob.rho0 + 2.0 * dr * c_old) / disc.tau
    dphi, dK, duin = theta_jacobians(prob, grid, theta)
    grad = dphi @ g_phi + dK @ g_K
    grad[12] = g_uin * duin
    return res.qoi, grad


def fd_gradient(prob, grid, theta, h=1e-6, opts: H.SolveOptions | None = None, comps=range(13)):
    """Central finite differences of Q with an absolute step h per component."""
    opts = opts or H.SolveOptions(stagnate=True)
    theta = np.asarray(theta, dtype=np.float64)
    g = np.zeros(13)
    for k in comps:
        tp = theta.copy(); tp[k] += h
        tm = theta.copy(); tm[k] -= h
        g[k] = (H.solve_sample(prob, grid, tp, opts).qoi - H.solve_sample(prob, grid, tm, opts).qoi) / (2 * h)
    return g
