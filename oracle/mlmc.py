"""Multilevel Monte Carlo estimator (paper section 3) -- TEST INFRASTRUCTURE ONLY.

  Y_l^(i) = g_l^(i) - g_{l-1}^(i), same random input on both grids, g_{-1} = 0
  estimate of E[g_L] = sum_l mean_i Y_l^(i)                     (eqs. EgL and A)
  V_l = unbiased sample variance of Y_l,  Var[Y] = sum_l V_l / m_l  (eq. goal_variance)
  cost S = sum_l m_l s_l
  optimal m_l = 2 eps^-2 sqrt(V_l / s_l) sum_i sqrt(V_i s_i)       (eq. M_ell)
  optimal cost S = 2 eps^-2 (sum_l sqrt(V_l s_l))^2                 (eq. total_cost_MLMC)
  MSE = Var[Y] + bias^2                                            (eq. MSE)

Bias estimate (the workload refines by 2 per level, first-order scheme):
|E[g_L - g]| ~ |mean Y_L| / (2^alpha - 1).

Field statistics use piecewise-constant injection (each coarse cell copied to
its 2 x 2 children) and, for the variance field, the difference of unbiased
sample variances of the coupled fine/coarse fields on each level.
"""
from __future__ import annotations

import math
import numpy as np


def estimate(g_fine, g_coarse, alpha: float = 1.0):
    """g_fine[l]: array [m_l]; g_coarse[l]: array [m_l] or None for l = 0.

    Returns dict(mean, var_of_estimator, bias, rmse, V, Ymean).
    """
    L = len(g_fine) - 1
    Ymean, V = [], []
    for l in range(L + 1):
        y = np.asarray(g_fine[l], dtype=np.float64)
        if l > 0:
            y = y - np.asarray(g_coarse[l], dtype=np.float64)
        m = y.size
        mu = y.sum() / m
        Ymean.append(mu)
        V.append(((y - mu) ** 2).sum() / (m - 1) if m > 1 else 0.0)
    m = np.array([np.asarray(g).size for g in g_fine], dtype=np.float64)
    V = np.array(V)
    var_est = float(np.sum(V / m))
    bias = abs(Ymean[L]) / (2.0 ** alpha - 1.0) if L > 0 else 0.0
    return dict(mean=float(np.sum(Ymean)), var_of_estimator=var_est, bias=bias,
                rmse=math.sqrt(var_est + bias * bias), V=V, Ymean=np.array(Ymean))


def inject(field, times: int = 1):
    """Piecewise-constant coarse -> fine transfer of a [ny, nx] field (2 x 2 children)."""
    f = np.asarray(field)
    for _ in range(times):
        f = np.repeat(np.repeat(f, 2, axis=-2), 2, axis=-1)
    return f


def field_estimate(c_fine, c_coarse):
    """c_fine[l]: [m_l, ny_l, nx_l]; c_coarse[l]: [m_l, ny_{l-1}, nx_{l-1}] or None.

    Returns (mean_field, var_field) on the finest grid.
    """
    L = len(c_fine) - 1
    mean = None
    var = None
    for l in range(L + 1):
        f = np.asarray(c_fine[l], dtype=np.float64)
        m = f.shape[0]
        dm = f.mean(axis=0)
        dv = f.var(axis=0, ddof=1) if m > 1 else np.zeros_like(dm)
        if l > 0:
            cc = np.asarray(c_coarse[l], dtype=np.float64)
            dm = dm - inject(cc.mean(axis=0))
            dv = dv - inject(cc.var(axis=0, ddof=1) if m > 1 else np.zeros_like(cc[0]))
        dm = inject(dm, L - l)
        dv = inject(dv, L - l)
        mean = dm if mean is None else mean + dm
        var = dv if var is None else var + dv
    return mean, var


def optimal_samples(V, s, eps):
    """m_l = ceil(2 eps^-2 sqrt(V_l/s_l) sum_i sqrt(V_i s_i)) and the model costs."""
    V = np.asarray(V, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    tot = np.sum(np.sqrt(V * s))
    m_real = 2.0 / eps ** 2 * np.sqrt(V / s) * tot
    m = np.ceil(m_real).astype(np.int64)
    return dict(m=m, m_real=m_real, cost=float(np.sum(m * s)),
                cost_opt=float(2.0 / eps ** 2 * tot ** 2))


def estimate_series(s_fine, s_coarse, alpha: float = 1.0):
    """Time-resolved QoIs: estimate() at every common time point and QoI.

    s_fine[l]: [m_l, r_l, nq] (level l's series after each of its r_l steps); s_coarse[l]:
    [m_l, r_{l-1}, nq] on the coarse partner's time grid, None for l = 0.  The common times
    are t_k = (k + 1) T / r_0: entry (k + 1) r_l / r_0 - 1 of level l's series.
    Returns dict(mean, var_of_estimator [r_0, nq], Ymean, V [L+1, r_0, nq]).
    """
    L = len(s_fine) - 1
    r0, nq = np.asarray(s_fine[0]).shape[1:]
    mean = np.zeros((r0, nq)); var = np.zeros((r0, nq))
    Ym = np.zeros((L + 1, r0, nq)); V = np.zeros((L + 1, r0, nq))
    for k in range(r0):
        for q in range(nq):
            gf, gc = [], []
            for l in range(L + 1):
                f = np.asarray(s_fine[l])
                gf.append(f[:, (k + 1) * (f.shape[1] // r0) - 1, q])
                if l == 0:
                    gc.append(None)
                else:
                    c = np.asarray(s_coarse[l])
                    gc.append(c[:, (k + 1) * (c.shape[1] // r0) - 1, q])
            e = estimate(gf, gc, alpha)
            mean[k, q], var[k, q] = e["mean"], e["var_of_estimator"]
            Ym[:, k, q], V[:, k, q] = e["Ymean"], e["V"]
    return dict(mean=mean, var_of_estimator=var, Ymean=Ym, V=V)


def fit_rate(levels, values):
    """values ~ c 2^(slope l): least-squares line through (l, log2 value); returns (slope, c)."""
    x = np.asarray(levels, dtype=np.float64)
    y = np.log2(np.asarray(values, dtype=np.float64))
    slope, icpt = np.polyfit(x, y, 1)
    return float(slope), float(2.0 ** icpt)


def plan(Ymean_abs, V, s, eps, E0, max_level):
    """Adaptive MLMC plan from pilot statistics on levels 0..Lp (section 3, eqs. num_levels
    and scaled_m_l_S; this hierarchy refines by 2 per level, so powers of 2 replace the
    paper's powers of 4).

    |E Y_l| = c1 2^(-alpha l) and V_l = c2 2^(-beta l) fitted over l = 1..Lp, the cost
    s_l = c3 2^(gamma l) over l = 0..Lp.  The bias of stopping at level L is the geometric
    tail sum_{l > L} |E Y_l| = c1 2^(-alpha L) / (2^alpha - 1); L is the smallest level in
    [1, max_level] where it is at most eps E0 / sqrt(2) (half the mean-square error budget),
    else max_level.  m_l = ceil(2 eps^-2 E0^-2 sqrt(V_l/s_l) sum_i sqrt(V_i s_i)) (eq.
    scaled_m_l_S), with the pilot's V_l and s_l for l <= Lp and the fitted laws beyond.
    mc_cost = 2 eps^-2 E0^-2 s_L V_0 is the cost of plain Monte Carlo at level L for the same
    accuracy (section 5, Test B4).
    """
    Lp = len(V) - 1
    sa, c1 = fit_rate(range(1, Lp + 1), Ymean_abs[1:])
    sb, c2 = fit_rate(range(1, Lp + 1), V[1:])
    gamma, c3 = fit_rate(range(0, Lp + 1), s)
    alpha, beta = -sa, -sb
    if not alpha > 0:
        raise ValueError("no weak convergence in the pilot")
    L = max_level
    for l in range(1, max_level + 1):
        if c1 * 2.0 ** (-alpha * l) / (2.0 ** alpha - 1.0) <= eps * E0 / math.sqrt(2.0):
            L = l
            break
    Vx = [V[l] if l <= Lp else c2 * 2.0 ** (-beta * l) for l in range(L + 1)]
    sx = [s[l] if l <= Lp else c3 * 2.0 ** (gamma * l) for l in range(L + 1)]
    tot = sum(math.sqrt(v * c) for v, c in zip(Vx, sx))
    m = [int(math.ceil(2.0 / (eps * E0) ** 2 * math.sqrt(v / c) * tot)) for v, c in zip(Vx, sx)]
    # section 5, Test B4: plain Monte Carlo at level L for the same accuracy, with the
    # pilot's Var g_0 standing in for Var g_L
    mc_cost = 2.0 / (eps * E0) ** 2 * sx[L] * V[0]
    return dict(L=L, m=m, cost=float(sum(mi * c for mi, c in zip(m, sx))), alpha=alpha, beta=beta, gamma=gamma,
                c1=c1, c2=c2, c3=c3, mc_cost=float(mc_cost))
