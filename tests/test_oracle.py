"""Pins of the CPU oracle against what the paper and the mathematics fix (CPU only).

Every check here is independent of the oracle's own formulas: closed forms,
invariants, brute force, library routines or numbers printed in the paper.
"""
import math
import os

import numpy as np
import pytest
from scipy import integrate, special

from henry_inputs import draw_theta, level_grid
from oracle import adjoint as A
from oracle import henry as H
from oracle import kl as KL
from oracle import mlmc as M

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _table(name):
    rows = []
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append(line.split())
    return rows


# ---------------------------------------------------------------- constants
def test_table1_constants_and_kozeny_carman():
    """Table 1 values; the mean permeability is Kozeny-Carman of the mean porosity (eq. e_perm_Kozeny_Carman)."""
    t = {r[0]: float(r[1]) for r in _table("paper_table1.txt")}
    pr = H.Problem()
    assert pr.phi_mean == t["phi_mean"]
    assert pr.Dm == pytest.approx(t["D"], rel=1e-12)
    assert pr.K_mean == t["K_hat"]
    assert pr.rho0 == t["rho0"] and pr.mu == t["mu"]
    # the studied workload rounds rho1 to 1025 (Table 1 prints 1024.99)
    assert abs(pr.rho1 - t["rho1"]) < 0.011
    kc = t["kappa_KC"] * t["phi_mean"] ** 3 / (1.0 - t["phi_mean"] ** 2)
    assert kc == pytest.approx(t["K_hat"], rel=1e-6)


# ---------------------------------------------------------------- KL basis
def test_kl_roots_satisfy_transcendental_equations():
    for a in (1.0, 0.5):
        c = 2.0
        for w, par, lam, _ in KL.roots_1d(a, 0.5, 10):
            if par == 0:
                r = (c * math.cos(w * a) - w * math.sin(w * a)) / max(c, w)
            else:
                r = (w * math.cos(w * a) + c * math.sin(w * a)) / max(c, w)
            assert abs(r) < 1e-14
            assert lam == pytest.approx(2 * c / (w * w + c * c), rel=1e-15)


def test_kl_1d_orthonormal_and_eigen_by_quadrature():
    """f is an eigenfunction: int exp(-|s-t|/b) f(t) dt = lam f(s), checked by adaptive quadrature."""
    a, b = 1.0, 0.5
    modes = KL.roots_1d(a, b, 6)
    for i, mi in enumerate(modes):
        for j, mj in enumerate(modes):
            v, _ = integrate.quad(lambda s: KL.eval_1d(mi, s, 0.0) * KL.eval_1d(mj, s, 0.0), -a, a, limit=200)
            assert abs(v - (1.0 if i == j else 0.0)) < 1e-10
        for s0 in (-0.7, 0.1, 0.9):
            lhs = sum(integrate.quad(lambda t: math.exp(-abs(s0 - t) / b) * KL.eval_1d(mi, t, 0.0), lo, hi,
                                     limit=200)[0] for lo, hi in ((-a, s0), (s0, a)))
            assert lhs == pytest.approx(mi[2] * KL.eval_1d(mi, s0, 0.0), abs=1e-10)


def test_kl_nystrom_and_trace():
    """Eigenvalues of the midpoint-rule kernel matrix approach the analytic ones; trace = domain length."""
    a, b, n = 1.0, 0.5, 2000
    s = -a + (np.arange(n) + 0.5) * (2 * a / n)
    Kmat = np.exp(-np.abs(s[:, None] - s[None, :]) / b) * (2 * a / n)
    ev = np.sort(np.linalg.eigvalsh(Kmat))[::-1][:6]
    lam = np.array([m[2] for m in KL.roots_1d(a, b, 6)])
    assert np.allclose(ev, lam, rtol=2e-5)
    # sum of all eigenvalues = int C(s, s) ds = 2a: the deficit of the partial sums decays like 1/N
    lam_many = np.array([m[2] for m in KL.roots_1d(a, b, 4000)])
    d1, d4 = 2 * a - lam_many[:1000].sum(), 2 * a - lam_many.sum()
    assert 0 < d4 < 5e-4 and 3.8 < d1 / d4 < 4.2


def test_kl_2d_orthonormal_on_fine_grid():
    kl = KL.KL2D()
    nx, ny = 512, 256
    x = (np.arange(nx) + 0.5) * 2.0 / nx
    y = -1.0 + (np.arange(ny) + 0.5) / ny
    X, Y = np.meshgrid(x, y)
    E = kl.table(X, Y).reshape(8, -1)
    G = E @ E.T * (2.0 / nx) * (1.0 / ny)
    assert np.abs(G - np.eye(8)).max() < 1e-5
    assert np.all(np.diff(kl.lam) <= 0)


def test_fields_theta_zero_and_ranges():
    pr = H.Problem()
    g = H.Grid(*level_grid(2))
    phi, K, u = H.sample_fields(pr, g, np.zeros(13))
    assert np.all(phi == 0.35) and u == pr.q_in
    assert np.abs(K / pr.K_mean - 1.0).max() < 1e-15   # exp(ln K) rounds
    th = draw_theta(0, 64)
    for t in th:
        phi, K, u = H.sample_fields(pr, g, t)
        assert 0.2 < phi.min() and phi.max() < 0.5
        assert u == pytest.approx(6.6e-5 * (1 + 0.1 * t[12]))


# ---------------------------------------------------------------- discrete operator
def _some_state(ns=3, grid=(16, 8, 12), seed=7):
    pr = H.Problem()
    g = H.Grid(*grid)
    th = draw_theta(seed, 2)[1]
    phi, K, u = H.sample_fields(pr, g, th)
    d = H.Discretisation(pr, g, phi, K, u)
    r = H.solve_sample(pr, g, th, nsteps=ns, keep_states=True)
    return pr, g, d, r


def test_jacobian_matches_finite_differences_of_residual():
    pr, g, d, r = _some_state()
    p, c = r.states[-1]
    c_old = r.states[-2][1]
    rng = np.random.default_rng(0)
    p = p + rng.normal(size=p.shape) * 10.0
    c = c + rng.normal(size=c.shape) * 0.01
    J = d.jacobian(p, c).toarray()
    n = d.nc
    for k in range(0, 2 * n, 7):
        e = 1e-6 if k % 2 else 1e-2
        pp, cp, pm, cm = p.copy(), c.copy(), p.copy(), c.copy()
        if k % 2:
            cp[k // 2] += e; cm[k // 2] -= e
        else:
            pp[k // 2] += e; pm[k // 2] -= e
        a1, b1 = d.residual(pp, cp, c_old)
        a0, b0 = d.residual(pm, cm, c_old)
        col = np.empty(2 * n); col[0::2] = (a1 - a0) / (2 * e); col[1::2] = (b1 - b0) / (2 * e)
        assert np.abs(col - J[:, k]).max() <= 1e-8 * np.abs(J).max()


def test_hydrostatic_seawater_is_exact_steady_state():
    """c = 1 everywhere, no recharge, c_left = 1: p = -rho1 g y and u = 0 to round-off."""
    pr = H.Problem(q_in=0.0, c_left=1.0)
    g = H.Grid(32, 16, 48)
    phi, K, u = H.sample_fields(pr, g, draw_theta(3, 1)[0])
    d = H.Discretisation(pr, g, phi, K, u)
    _, Y = H.cell_centres(pr, g)
    p_h = (-pr.rho1 * pr.g * Y).ravel()
    c1 = np.ones(d.nc)
    Rp, Rc = d.residual(p_h, c1, c1)
    scale = pr.rho0 * pr.K_mean / pr.mu * pr.rho1 * pr.g * (1.0 / 16)
    assert np.abs(Rp).max() < 1e-12 * scale and np.abs(Rc).max() < 1e-12 * scale
    f = d._face(p_h, c1, d.nP, d.nQ, True)
    assert np.abs(f["u"]).max() < 1e-15
    # Newton from a perturbed pressure returns to it
    p0 = p_h + 50.0 * np.sin(np.arange(d.nc))
    p, c, its, ok = H.newton_step(d, p0, c1, c1, H.SolveOptions(newton_tol=1e-12))
    assert ok and np.abs(p - p_h).max() < 1e-9 * pr.rho1 * pr.g and np.abs(c - 1).max() < 1e-12


def test_hydrostatic_fresh_water():
    pr = H.Problem(q_in=0.0, rho1=1000.0)
    g = H.Grid(32, 16, 48)
    phi, K, u = H.sample_fields(pr, g, draw_theta(3, 1)[0])
    d = H.Discretisation(pr, g, phi, K, u)
    _, Y = H.cell_centres(pr, g)
    p_h = (-pr.rho0 * pr.g * Y).ravel()
    z = np.zeros(d.nc)
    p, c, its, ok = H.newton_step(d, p_h + 10.0, z, z, H.SolveOptions(newton_tol=1e-12))
    assert ok and np.abs(p - p_h).max() < 1e-9 * pr.rho0 * pr.g and np.abs(c).max() < 1e-14


def _ogata_banks(x, t, v, D):
    """1-D advection-diffusion, c(0, t) = 1, c(x, 0) = 0 on x > 0 (Ogata & Banks 1961)."""
    s = 2.0 * np.sqrt(D * t)
    z1 = (x - v * t) / s
    z2 = (x + v * t) / s
    return 0.5 * (special.erfc(z1) + np.exp(v * x / D - z2 * z2) * special.erfcx(z2))


def test_constant_density_reduces_to_advection_diffusion():
    """rho1 = rho0, theta = 0, c_left = 1: y-independent, first-order convergence to the erfc solution
    (paper eq. 1st_ord_conv), and Richardson extrapolation of two grids converges at second order."""
    pr = H.Problem(rho1=1000.0, c_left=1.0, T=3600.0)
    v = pr.q_in / pr.phi_mean
    sols, errs = {}, []
    for nx, nsteps in ((100, 36), (200, 72), (400, 144)):
        g = H.Grid(nx, 2, nsteps)
        r = H.solve_sample(pr, g, np.zeros(13), H.SolveOptions(newton_tol=1e-12))
        c = r.c.reshape(2, nx)
        assert np.abs(c[0] - c[1]).max() < 1e-12
        x = (np.arange(nx) + 0.5) * 2.0 / nx
        m = x < 1.5                     # away from the outflow boundary (semi-infinite solution)
        errs.append(np.abs(c[0] - _ogata_banks(x, pr.T, v, pr.Dm))[m].max())
        sols[nx] = c[0]
    assert 1.7 < errs[0] / errs[1] < 2.3 and 1.7 < errs[1] / errs[2] < 2.3
    rich = []
    for nc in (100, 200):
        cf = sols[2 * nc]
        x = (np.arange(nc) + 0.5) * 2.0 / nc
        m = x < 1.5
        extrap = 2.0 * 0.5 * (cf[0::2] + cf[1::2]) - sols[nc]
        rich.append(np.abs(extrap - _ogata_banks(x, pr.T, v, pr.Dm))[m].max())
    assert rich[0] < errs[0] / 8 and 3.0 < rich[0] / rich[1] < 4.5


def test_mass_balance_bounds_and_convergence_level0():
    """Conservation (storage change = boundary fluxes) and c in [0, 1] on real level-0 samples."""
    pr = H.Problem()
    g = H.Grid(*level_grid(0))
    th = draw_theta(0, 16)
    for s in (0, 5):
        r = H.solve_sample(pr, g, th[s])
        assert r.converged
        assert r.max_fluid_defect < 1e-10 and r.max_salt_defect < 1e-10
        assert -1e-10 <= r.c_min and r.c_max <= 1 + 1e-10
        assert 0 < r.qoi < 1025.0


def test_dirichlet_right_variant_keeps_bounds():
    pr = H.Problem(right_c_dirichlet=True)
    g = H.Grid(32, 16, 12)
    r = H.solve_sample(pr, g, draw_theta(0, 2)[1])
    assert r.converged and r.max_salt_defect < 1e-10
    assert -1e-10 <= r.c_min and r.c_max <= 1 + 1e-10


# ------------------------------------------------ the paper's own model (section 4)
def test_paper_porosity_at_points_where_most_terms_vanish():
    """eq. poro_2levels at points where all but one or two terms vanish (values by hand):
    x = 0, 1, 2 put cos(pi x/2) at 1, 0, -1; y = -0.5 and y = -0.25 put sin(2 pi y) at 0 and
    -1 and sin(32 pi y) at 0; x = 0, 0.5, 1 put sin(64 pi x) at 0; y < -0.8 selects the
    second layer factor 1.2 (1 + 0.2 xi_1)."""
    P = lambda x, y, a, b: float(H.paper_porosity(np.array(x), np.array(y), a, b))
    assert P(0.0, -0.5, 0.0, 1.0) == pytest.approx(0.35 * 1.15, rel=1e-14)    # xi_2 cos(pi x/2)
    assert P(2.0, -0.5, 0.0, 1.0) == pytest.approx(0.35 * 0.85, rel=1e-14)
    assert P(1.0, -0.25, 0.0, 1.0) == pytest.approx(0.35 * 1.15, rel=1e-14)   # -xi_2 sin(2 pi y)
    assert P(1.0, -0.25, 0.0, -1.0) == pytest.approx(0.35 * 0.85, rel=1e-14)
    assert P(0.0, -0.5, 1.0, 0.0) == pytest.approx(0.35 * 1.15, rel=1e-14)    # xi_1 cos(2 pi x)
    assert P(0.5, -0.5, 1.0, 0.0) == pytest.approx(0.35 * 0.85, rel=1e-14)
    assert P(1.0, -0.9, 1.0, 0.0) == pytest.approx(0.35 * 1.44 * 1.15, rel=1e-14)  # layer: 1.2 * 1.2
    assert P(1.0, -0.9, -1.0, 0.0) == pytest.approx(0.35 * 0.96 * 0.85, rel=1e-14)
    assert P(1.0, -0.7, 1.0, 0.0) == pytest.approx(0.35 * 1.15, rel=1e-14)
    # small scales: sin(64 pi x) = 1 at x = 1/128 + k/32, sin(32 pi y) = 1 at y = -63/64
    x = 0.5 + 1.0 / 128.0   # cos(2 pi x) = -cos(pi/64)
    assert P(x, -0.5, 1.0, 0.0) == pytest.approx(0.35 * (1.0 - 0.15 * math.cos(math.pi / 64)) * 1.2, rel=1e-14)
    # y = -33/64: sin(32 pi y) = sin(-16.5 pi) = -1, sin(2 pi y) = sin(pi/32)
    assert P(1.0, -33.0 / 64.0, 0.0, 1.0) == pytest.approx(0.35 * (1.0 - 0.15 * math.sin(math.pi / 32)) * 0.8, rel=1e-14)


def test_paper_fields_theta_zero_two_layers_and_kozeny_carman():
    """theta = 0: phi = 0.35 above y = -0.8 and 0.42 below; K there is Kozeny-Carman of phi,
    which at 0.35 is Table 1's K (so kappa_KC and K_hat agree), on every cell-centred grid."""
    pr = H.paper_problem()
    t1 = {r[0]: float(r[1]) for r in _table("paper_table1.txt")}
    assert pr.kappa_kc == t1["kappa_KC"]
    for lev in (0, 2):
        g = H.Grid(*level_grid(lev))
        phi, K, u = H.sample_fields(pr, g, np.zeros(13))
        _, Y = H.cell_centres(pr, g)
        np.testing.assert_allclose(phi[Y > -0.8], 0.35, rtol=1e-15)
        np.testing.assert_allclose(phi[Y < -0.8], 0.42, rtol=1e-15)
        np.testing.assert_allclose(K[Y > -0.8], t1["K_hat"], rtol=1e-6)
        np.testing.assert_allclose(K[Y < -0.8], t1["kappa_KC"] * 0.42 ** 3 / (1 - 0.42 ** 2), rtol=1e-6)
        assert u == pytest.approx(6.6e-5)
    th = np.zeros(13); th[0], th[1] = 0.7, -0.4
    g = H.Grid(*level_grid(2))
    phi2, _, _ = H.sample_fields(pr, g, th)
    assert 0.11 < phi2.min() and phi2.max() < 0.92     # bounds of C0 C1 C2 for |xi| <= 1
    # q_in with xi_3: 6.6e-5 (1 + 0.5 xi_3)
    th[12] = -0.6
    assert H.sample_fields(pr, g, th)[2] == pytest.approx(6.6e-5 * 0.7, rel=1e-15)


def test_recharge_pressure_closed_form_each_step():
    """Constant density (rho1 = rho0), uniform phi and K (KL model, theta = 0) with the
    periodic recharge: the flow is incompressible and one-dimensional, so after the step
    ending at t_n the pressure is exactly p = -rho0 g y + mu u_in(t_n) (Lx - x) / K with
    u_in(t) = 6.6e-5 (1 + 0.5 zeta)(1 + sin(pi t / 40)) -- boundary data at the new time
    level (implicit Euler), the two-point flux being exact for a linear profile."""
    pr = H.Problem(rho1=1000.0, q_in_amp=0.5, recharge_omega=np.pi / 40.0, T=130.0)
    g = H.Grid(8, 4, 13)
    th = np.zeros(13); th[12] = 0.4
    r = H.solve_sample(pr, g, th, keep_states=True)
    assert r.converged
    X, Y = H.cell_centres(pr, g)
    tau = pr.T / g.nsteps
    for n in range(1, g.nsteps + 1):
        u = 6.6e-5 * 1.2 * (1.0 + math.sin(math.pi * n * tau / 40.0))
        p_exact = -1000.0 * 9.81 * Y + 1e-3 * u * (2.0 - X) / 1.020408e-9
        np.testing.assert_allclose(r.states[n][0], p_exact.ravel(), rtol=1e-12, atol=1e-9 * 1000 * 9.81)
        assert np.abs(r.states[n][1]).max() == 0.0


def test_paper_model_balance_and_bounds_level0():
    """The paper's model (section 4, T = 6016 s) at level 0: per-step conservation with the
    time-dependent inflow, c in [0, 1], Newton converged."""
    pr = H.paper_problem()
    g = H.Grid(*level_grid(0))
    th = draw_theta(0, 4)
    for s in (0, 3):
        r = H.solve_sample(pr, g, th[s])
        assert r.converged
        assert r.max_fluid_defect < 1e-10 and r.max_salt_defect < 1e-10
        assert -1e-10 <= r.c_min and r.c_max <= 1 + 1e-10
        assert 0 < r.qoi < 1025.0


# ------------------------------------------------ time-resolved QoIs (section 5)
def test_series_qois_hand_values():
    """Q_S, Q_FW, Q_1..Q_15 (eqs. integral_s, integral_fw, integral_box) of simple fields, by
    hand: the boxes around y = -0.95 stick out below the domain (area 0.2 x 0.15), the others
    lie inside (0.2 x 0.2); x = 1 is a cell face on every level."""
    pr = H.Problem()
    for lev in (0, 2):
        g = H.Grid(*level_grid(lev))
        X, _ = H.cell_centres(pr, g)
        one = np.ones(g.nx * g.ny)
        np.testing.assert_allclose(H.series_qois(pr, g, one),
                                   [2050.0, 0.0] + [1025 * 0.03] * 5 + [1025 * 0.04] * 10, rtol=1e-13)
        np.testing.assert_allclose(H.series_qois(pr, g, 0.5 * one)[:2], [0.5 * 1012.5 * 2.0, 0.0], rtol=1e-13)
        np.testing.assert_allclose(H.series_qois(pr, g, 0.0 * one), [0.0, 2.0] + [0.0] * 15, atol=1e-13)
        right = (X > 1.0).astype(float).ravel()       # salt water right of x = 1
        want = [1025.0, 1.0] + sum(([0.0] + [1025 * a] * 4 for a in (0.03, 0.04, 0.04)), [])
        np.testing.assert_allclose(H.series_qois(pr, g, right), want, rtol=1e-13, atol=1e-12)


def test_series_qois_of_piecewise_constant_field_do_not_depend_on_the_grid():
    """The exact integral of a field constant on level-0 cells is the same when the field is
    represented on a finer grid (each coarse cell injected into its children): box overlaps
    that are partial on level 0 become whole fine cells."""
    pr = H.Problem()
    rng = np.random.default_rng(5)
    c0 = rng.random((16, 32))
    g0, g2 = H.Grid(*level_grid(0)), H.Grid(*level_grid(2))
    c2 = np.kron(c0, np.ones((4, 4)))
    np.testing.assert_allclose(H.series_qois(pr, g0, c0.ravel()), H.series_qois(pr, g2, c2.ravel()), rtol=1e-12)


def test_series_follow_the_solve():
    """The per-step series of a level-0 solve: the last step's salt mass over the whole domain
    bounds the salt mass in x > 1 (the QoI), all box masses are non-negative and bounded by
    the whole-domain mass, and the fresh-water area shrinks as the wedge enters."""
    pr = H.Problem()
    g = H.Grid(*level_grid(0))
    r = H.solve_sample(pr, g, draw_theta(0, 1)[0], series=True)
    s = r.series
    assert s.shape == (48, H.N_SERIES)
    assert s[-1, 0] >= r.qoi > 0
    assert (s[:, 2:] >= -1e-12).all() and (s[:, 2:].sum(axis=1) <= s[:, 0] + 1e-9).all()
    assert s[-1, 1] < s[0, 1] <= 2.0
    np.testing.assert_allclose(s[-1], H.series_qois(pr, g, r.c), rtol=0, atol=0)


# ---------------------------------------------------------------- MLMC
def test_mlmc_single_level_is_sample_mean_and_variance():
    rng = np.random.default_rng(3)
    g = rng.normal(size=37)
    e = M.estimate([g], [None])
    assert e["mean"] == pytest.approx(np.mean(g), rel=1e-14)
    assert e["V"][0] == pytest.approx(np.var(g, ddof=1), rel=1e-13)
    assert e["var_of_estimator"] == pytest.approx(np.var(g, ddof=1) / 37, rel=1e-13)


def test_mlmc_telescoping_identity():
    """Same inputs on every level: the telescoping sum collapses to the finest-level mean."""
    rng = np.random.default_rng(4)
    m = 50
    gl = [rng.normal(size=m) + l for l in range(4)]
    fine = [gl[0]] + [gl[l] for l in range(1, 4)]
    coarse = [None] + [gl[l - 1] for l in range(1, 4)]
    e = M.estimate(fine, coarse)
    assert e["mean"] == pytest.approx(np.mean(gl[3]), abs=1e-13)
    cf = [rng.normal(size=(m, 2 << l, 4 << l)) for l in range(3)]
    mean, var = M.field_estimate([cf[0], cf[1], cf[2]], [None, cf[0], cf[1]])
    assert np.allclose(mean, cf[2].mean(0), atol=1e-13)
    assert np.allclose(var, cf[2].var(0, ddof=1), atol=1e-12)


def test_injection_conserves_integrals():
    rng = np.random.default_rng(5)
    f = rng.normal(size=(4, 8))
    fi = M.inject(f, 2)
    assert fi.shape == (16, 32) and fi.sum() / 16 == pytest.approx(f.sum(), rel=1e-14)


def test_optimal_samples_formula_is_the_constrained_optimum():
    """eq. M_ell: Var[Y] = eps^2/2 at the real-valued optimum and no feasible perturbation is cheaper."""
    V = np.array([2.0, 0.4, 0.06, 0.01])
    s = np.array([1.0, 8.0, 64.0, 512.0])
    eps = 0.05
    o = M.optimal_samples(V, s, eps)
    mr = o["m_real"]
    assert np.sum(V / mr) == pytest.approx(eps ** 2 / 2, rel=1e-13)
    assert np.sum(mr * s) == pytest.approx(o["cost_opt"], rel=1e-13)
    rng = np.random.default_rng(0)
    for _ in range(200):
        m2 = mr * np.exp(0.2 * rng.normal(size=4))
        m2 *= np.sum(V / m2) / (eps ** 2 / 2)      # rescale onto the variance constraint
        assert np.sum(m2 * s) >= o["cost_opt"] * (1 - 1e-12)


def test_optimal_samples_reproduce_table3_eps_scaling():
    """Table 3: levels and costs at eps = 0.01 fix V_l up to a constant; eq. M_ell at eps = 0.007 then
    reproduces the printed m_l (within the ceiling), and Table 2's times give the printed MLMC cost."""
    t3 = {float(r[0]): r for r in _table("paper_table3.txt")}
    s = np.array([float(r[4]) for r in _table("paper_table2.txt")])
    m01 = np.array([float(x) for x in t3[0.01][4:8]])
    m007 = np.array([float(x) for x in t3[0.007][4:8]])
    kappa = 0.01 ** 2 / (2.0 * np.sum(m01 * s))
    V = kappa * m01 ** 2 * s
    o = M.optimal_samples(V, s, 0.007)
    r = (0.01 / 0.007) ** 2
    assert np.all(np.abs(o["m"] - m007) <= r + 1)
    for eps in (0.01, 0.007):
        m = np.array([float(x) for x in t3[eps][4:8]])
        assert np.sum(m * s) == pytest.approx(float(t3[eps][2]), rel=0.12)


@pytest.mark.slow
def test_series_estimate_is_the_scalar_estimator_at_each_common_time():
    """Level l's entry (k+1) r_l / r_0 - 1 is the common time t_k; a series whose values
    are the same at every step reproduces the scalar estimate at every time."""
    rng = np.random.default_rng(2)
    m = [30, 9, 4]
    g = [rng.normal(size=k) for k in m]
    gc = [None] + [g[l] + rng.normal(size=m[l]) * 0.1 for l in (1, 2)]
    ref = M.estimate(g, gc)
    r = [3 << l for l in range(3)]
    sf = [np.repeat(g[l][:, None, None], r[l], axis=1) * np.array([1.0, -2.0]) for l in range(3)]
    sc = [None] + [np.repeat(gc[l][:, None, None], r[l - 1], axis=1) * np.array([1.0, -2.0]) for l in (1, 2)]
    e = M.estimate_series(sf, sc)
    assert e["mean"].shape == (3, 2)
    np.testing.assert_allclose(e["mean"][:, 0], ref["mean"], rtol=1e-14)
    np.testing.assert_allclose(e["mean"][:, 1], -2 * ref["mean"], rtol=1e-14)
    np.testing.assert_allclose(e["var_of_estimator"][:, 1], 4 * ref["var_of_estimator"], rtol=1e-13)
    # entries off the common times are never read
    sf[2][:, 0::4, :] = np.nan
    sf[2][:, 1::4, :] = np.nan
    sf[2][:, 2::4, :] = np.nan
    assert np.isfinite(M.estimate_series(sf, sc)["mean"]).all()


def test_plan_recovers_exact_rates_and_levels():
    """Pilot data that follow the power laws exactly: the fit returns the rates; the level
    count follows the bias rule by hand; m_l is eq. M_ell at accuracy eps E0."""
    a, b, g = 1.0, 2.0, 3.0
    lv = np.arange(4)
    Ym = 1.0 * 2.0 ** (-a * lv)
    V = 0.5 * 2.0 ** (-b * lv)
    s = 0.25 * 2.0 ** (g * lv)
    p = M.plan(Ym, V, s, eps=0.01, E0=10.0, max_level=6)
    assert p["alpha"] == pytest.approx(a, rel=1e-12) and p["beta"] == pytest.approx(b, rel=1e-12)
    assert p["gamma"] == pytest.approx(g, rel=1e-12)
    assert p["c1"] == pytest.approx(1.0, rel=1e-12) and p["c2"] == pytest.approx(0.5, rel=1e-12)
    # bias 2^-L <= 0.01 * 10 / sqrt(2) = 0.0707: L = 4 (2^-3 = 0.125 is too large)
    assert p["L"] == 4
    Vx = 0.5 * 2.0 ** (-b * np.arange(5))
    sx = 0.25 * 2.0 ** (g * np.arange(5))
    want = M.optimal_samples(Vx, sx, 0.01 * 10.0)
    assert p["m"] == list(want["m"])
    # the bias target cannot be met below max_level
    assert M.plan(Ym, V, s, eps=1e-6, E0=1.0, max_level=5)["L"] == 5
    # Test B4's plain Monte Carlo cost at level L = 4 by hand: 2 (0.01 * 10)^-2 * s_4 * V_0
    # = 200 * 0.25 * 2^12 * 0.5
    assert p["mc_cost"] == pytest.approx(200.0 * 0.25 * 4096.0 * 0.5, rel=1e-12)
    # beta < gamma (as in the paper, beta ~ 1.7 < 3): the MLMC saving over plain MC grows as
    # the accuracy tightens (section 5 reports factors from about 30 to 3000)
    ratio = [M.plan(Ym, 0.5 * 2.0 ** (-1.7 * lv), s, eps=e, E0=10.0, max_level=12) for e in (0.03, 0.003, 0.0003)]
    ratio = [q["mc_cost"] / q["cost"] for q in ratio]
    assert 1.0 < ratio[0] < ratio[1] < ratio[2] and ratio[2] > 1000.0


def test_mlmc_agrees_with_plain_mc_on_tiny_levels():
    pr = H.Problem(T=7200.0)
    g0, g1 = H.Grid(8, 4, 6), H.Grid(16, 8, 12)
    th_mc = draw_theta(11, 48, level=1)
    q_mc = np.array([H.solve_sample(pr, g1, t).qoi for t in th_mc])
    th0 = draw_theta(12, 96, level=0)
    th1 = draw_theta(12, 16, level=1)
    q0 = np.array([H.solve_sample(pr, g0, t).qoi for t in th0])
    q1f = np.array([H.solve_sample(pr, g1, t).qoi for t in th1])
    q1c = np.array([H.solve_sample(pr, g0, t).qoi for t in th1])
    e = M.estimate([q0, q1f], [None, q1c])
    sd = math.sqrt(e["var_of_estimator"] + np.var(q_mc, ddof=1) / q_mc.size)
    assert abs(e["mean"] - q_mc.mean()) < 3 * sd
    assert e["V"][1] < 0.25 * e["V"][0]


# ---------------------------------------------------------------- adjoint
def test_adjoint_matches_central_differences():
    pr = H.Problem()
    g = H.Grid(16, 8, 12)
    th = draw_theta(7, 2)[1]
    q, ga = A.adjoint_gradient(pr, g, th)
    gf = A.fd_gradient(pr, g, th, h=1e-6)
    assert np.abs(ga - gf).max() <= 1e-6 * np.abs(gf).max()


def test_paper_model_adjoint_matches_central_differences():
    """The paper's model (section 4): xi_1, xi_2 act through eq. poro_2levels and the
    Kozeny-Carman permeability, xi_3 through the periodic recharge, whose time factor
    differs from step to step (dropping it fails the xi_3 component).  The other ten
    components do not enter the model: their adjoint gradient is exactly zero."""
    pr = H.paper_problem(T=6016.0 * 12 / 48)
    g = H.Grid(16, 8, 12)
    th = draw_theta(8, 3)[2]
    q, ga = A.adjoint_gradient(pr, g, th)
    gf = A.fd_gradient(pr, g, th, h=1e-6, comps=(0, 1, 12))
    for k in (0, 1, 12):
        assert abs(ga[k] - gf[k]) <= 1e-6 * np.abs(gf).max(), (k, ga[k], gf[k])
    assert np.all(ga[2:12] == 0.0)
    assert min(abs(ga[0]), abs(ga[1]), abs(ga[12])) > 1e-3 * np.abs(ga).max()


def test_paper_model_adjoint_taylor_remainder_is_second_order():
    """|Q(theta + e d) - Q(theta) - e g.d| shrinks by 4 when e halves, along a direction in
    the three parameters of the paper's model."""
    pr = H.paper_problem(T=6016.0 * 8 / 48)
    g = H.Grid(16, 8, 8)
    th = draw_theta(10, 1)[0]
    q, ga = A.adjoint_gradient(pr, g, th)
    d = np.zeros(13)
    d[[0, 1, 12]] = np.random.default_rng(2).normal(size=3)
    opts = H.SolveOptions(stagnate=True)
    rem = []
    for eps in (1e-2, 5e-3, 2.5e-3):
        qe = H.solve_sample(pr, g, th + eps * d, opts).qoi
        rem.append(abs(qe - q - eps * ga @ d))
    assert 3.0 < rem[0] / rem[1] < 5.0 and 3.0 < rem[1] / rem[2] < 5.0


def test_adjoint_taylor_remainder_is_second_order():
    pr = H.Problem()
    g = H.Grid(16, 8, 8)
    th = draw_theta(9, 1)[0]
    q, ga = A.adjoint_gradient(pr, g, th)
    d = np.random.default_rng(1).normal(size=13)
    opts = H.SolveOptions(stagnate=True)
    rem = []
    for eps in (1e-2, 5e-3, 2.5e-3):
        qe = H.solve_sample(pr, g, th + eps * d, opts).qoi
        rem.append(abs(qe - q - eps * ga @ d))
    assert 3.0 < rem[0] / rem[1] < 5.0 and 3.0 < rem[1] / rem[2] < 5.0


# ---------------------------------------------------------------- pins of single branches
def test_qoi_salt_mass_hand_values():
    """Q = sum over the cells whose centre lies in x > 1 of c rho(c) |cell| (section 5, eq. integral_s:
    the mass of salt is c rho, without porosity).  The part x > 1 of [0,2]x[-1,0] has area 1 m^2."""
    pr = H.Problem()
    for lev in (0, 2):
        g = H.Grid(*level_grid(lev))
        n = g.nx * g.ny
        X, _ = H.cell_centres(pr, g)
        assert H.qoi_salt_mass(pr, g, np.ones(n)) == pytest.approx(1025.0, rel=1e-13)          # c = 1: rho1 * 1 m^2
        assert H.qoi_salt_mass(pr, g, np.full(n, 0.5)) == pytest.approx(0.5 * 1012.5, rel=1e-13)
        assert H.qoi_salt_mass(pr, g, (X < 1.0).astype(float).ravel()) == 0.0                  # salt only in x < 1
        band = ((X > 1.0) & (X < 1.5)).astype(float).ravel()                                   # 1 <= x <= 1.5
        assert H.qoi_salt_mass(pr, g, band) == pytest.approx(1025.0 * 0.5, rel=1e-13)


def _nystrom_modes(L, b, n):
    """1-D eigenpairs of exp(-|s - t|/b) on an interval of length L by the midpoint-rule Nystrom
    method (numpy eigh; independent of the closed-form roots): eigenvalues and eigenfunction
    values at the n midpoints, L2-normalised, sign fixed as the analytic modes fix it (even modes
    positive at the centre, odd modes positive just right of it).  Returns [(lam, f, parity)]."""
    h = L / n
    s = (np.arange(n) + 0.5) * h
    lam, V = np.linalg.eigh(np.exp(-np.abs(s[:, None] - s[None, :]) / b) * h)
    out = []
    for k in np.argsort(lam)[::-1][:12]:
        f = V[:, k] / np.sqrt(h)
        even = np.abs(f - f[::-1]).max() < 1e-6 * np.abs(f).max()
        if f[n // 2] < 0:            # centre value (even) or first value right of the centre (odd)
            f = -f
        out.append((lam[k], f, 0 if even else 1))
    return out


def test_kl_fields_single_coefficients_against_nystrom_modes():
    """theta with one non-zero slot: xi_k = 1 must give phi = 0.35 (1 + 0.2 sqrt(lam_k) e_k), eta_k = 1
    ln K = ln K_hat + 0.5 sqrt(lam_k) e_k, zeta = 1 the inflow 6.6e-5 * 1.1; lam_k, e_k from an
    independent Nystrom discretisation of the separable exponential covariance (2-D pairs sorted by
    lam, descending), at the cell centres of a 1024 x 512 grid (the midpoint nodes).  This pins the
    slot -> mode map, the sqrt(lam) weights and the two amplitudes."""
    pr = H.Problem()
    g = H.Grid(1024, 512, 1)
    mx = _nystrom_modes(2.0, 0.5, 1024)
    my = _nystrom_modes(1.0, 0.5, 512)
    pairs = sorted(((a[0] * c[0], ix, iy) for ix, a in enumerate(mx) for iy, c in enumerate(my)),
                   key=lambda t: (-t[0], t[1]))[:8]
    E = [np.outer(my[iy][1], mx[ix][1]) for _, ix, iy in pairs]        # [ny, nx], rows bottom to top
    lam = np.array([p[0] for p in pairs])
    assert lam == pytest.approx([0.445499, 0.248790, 0.151538, 0.133054, 0.084627, 0.076935, 0.060876,
                                 0.048623], rel=3e-4)
    for k in range(4):
        th = np.zeros(13)
        th[k] = 1.0
        phi, K, u = H.sample_fields(pr, g, th)
        want = 0.35 * (1.0 + 0.2 * np.sqrt(lam[k]) * E[k])
        assert np.abs(phi - want).max() <= 2e-4 * np.abs(want - 0.35).max(), k
        assert np.abs(K / pr.K_mean - 1.0).max() < 1e-15 and u == pr.q_in     # exp(ln K) rounds
    for k in range(8):
        th = np.zeros(13)
        th[4 + k] = 1.0
        phi, K, u = H.sample_fields(pr, g, th)
        want = 0.5 * np.sqrt(lam[k]) * E[k]
        assert np.abs(np.log(K / pr.K_mean) - want).max() <= 2e-4 * np.abs(want).max(), k
        assert np.all(phi == 0.35) and u == pr.q_in
    th = np.zeros(13)
    th[12] = 1.0
    phi, K, u = H.sample_fields(pr, g, th)
    assert u == pytest.approx(6.6e-5 * 1.1, rel=1e-15) and np.all(phi == 0.35)
    # all slots at once: superposition of the single-mode fields
    th = draw_theta(11, 1)[0]
    phi, K, u = H.sample_fields(pr, g, th)
    sp = sum(np.sqrt(lam[k]) * th[k] * E[k] for k in range(4))
    sk = sum(np.sqrt(lam[k]) * th[4 + k] * E[k] for k in range(8))
    assert np.abs(phi - 0.35 * (1 + 0.2 * sp)).max() <= 1e-3 * np.abs(0.35 * 0.2 * sp).max()
    assert np.abs(np.log(K / pr.K_mean) - 0.5 * sk).max() <= 1e-3 * np.abs(0.5 * sk).max()


def test_mlmc_bias_and_rmse_on_a_two_level_hand_example():
    """eqs. A, goal_variance, MSE and the bias estimate |mean Y_L| / (2^alpha - 1), by hand:
    Y_0 = (1, 2, 3): mean 2, V_0 = 1; Y_1 = (5, 7) - (4, 5) = (1, 2): mean 1.5, V_1 = 0.5.
    mean = 3.5, Var = 1/3 + 0.5/2 = 7/12; alpha = 1: bias 1.5, rmse = sqrt(7/12 + 2.25);
    alpha = 2: bias 0.5, rmse = sqrt(7/12 + 0.25)."""
    e = M.estimate([np.array([1.0, 2.0, 3.0]), np.array([5.0, 7.0])], [None, np.array([4.0, 5.0])], alpha=1.0)
    assert e["mean"] == pytest.approx(3.5, rel=1e-15)
    assert e["V"] == pytest.approx([1.0, 0.5], rel=1e-15)
    assert e["var_of_estimator"] == pytest.approx(7.0 / 12.0, rel=1e-15)
    assert e["bias"] == pytest.approx(1.5, rel=1e-15)
    assert e["rmse"] == pytest.approx(math.sqrt(7.0 / 12.0 + 2.25), rel=1e-15)
    e = M.estimate([np.array([1.0, 2.0, 3.0]), np.array([5.0, 7.0])], [None, np.array([4.0, 5.0])], alpha=2.0)
    assert e["bias"] == pytest.approx(0.5, rel=1e-15)
    assert e["rmse"] == pytest.approx(math.sqrt(7.0 / 12.0 + 0.25), rel=1e-15)


def test_residual_by_hand_on_a_three_by_two_grid():
    """Residual of one implicit-Euler step on 3 x 2 unit cells ([0,3]x[-2,0], tau = 100 s), evaluated
    face by face with scalar arithmetic from the discrete balance laws (section 2.1: fluid and salt
    mass, Darcy with rho(c) g on vertical faces, D = phi Dm).  The state hits every branch: the left
    inflow with its Dirichlet diffusion, a right-side inflow cell (rho1 and c = 1 enter) and a
    right-side outflow cell, upwinding in both directions on east and north faces, gravity on the
    north faces, harmonic K."""
    pr = H.Problem(Lx=3.0, Ly=2.0, T=1000.0)
    g = H.Grid(3, 2, 10)
    rho0, dr, mu, grav, Dm, tau = 1000.0, 25.0, 1e-3, 9.81, pr.Dm, 100.0
    phi = np.array([[0.30, 0.35, 0.40], [0.25, 0.30, 0.45]])           # [j, i], j = 0 is the bottom row
    K = np.array([[1e-9, 2e-9, 1e-9], [3e-9, 1e-9, 2e-9]])
    u_in = 1.2e-4
    y = np.array([-1.5, -0.5])
    pb = -1025.0 * grav * y                                             # right boundary pressure per row
    c = np.array([[0.1, 0.4, 0.8], [0.2, 0.5, 0.9]])
    c_old = np.array([[0.0, 0.3, 0.7], [0.1, 0.6, 0.8]])
    # bottom row: p falls eastward except into the right inflow cell; top row rises at the end
    p = np.array([[pb[0] + 30.0, pb[0] + 10.0, pb[0] - 20.0],
                  [pb[1] - 80.0, pb[1] - 60.0, pb[1] + 40.0]])
    R = np.zeros((2, 2, 3))                                             # [p or c][j][i]
    rho = lambda v: rho0 + dr * v
    branches = set()
    for j in range(2):
        for i in range(3):
            R[0, j, i] += phi[j, i] * (rho(c[j, i]) - rho(c_old[j, i])) / tau
            R[1, j, i] += phi[j, i] * (rho(c[j, i]) * c[j, i] - rho(c_old[j, i]) * c_old[j, i]) / tau
    faces = [((j, i), (j, i + 1), False) for j in range(2) for i in range(2)] + \
            [((0, i), (1, i), True) for i in range(3)]
    for P, Q, north in faces:
        Kf = 2.0 * K[P] * K[Q] / (K[P] + K[Q])
        rf = 0.5 * (rho(c[P]) + rho(c[Q]))
        u = -(Kf / mu) * ((p[Q] - p[P]) / 1.0 + (rf * grav if north else 0.0))
        F = rf * u * 1.0
        cup = c[P] if F >= 0 else c[Q]
        branches.add(("north" if north else "east", F >= 0))
        G = F * cup - rf * 0.5 * (phi[P] + phi[Q]) * Dm * (c[Q] - c[P])
        R[0][P] += F; R[0][Q] -= F
        R[1][P] += G; R[1][Q] -= G
    for j in range(2):
        F = -rho0 * u_in * 1.0                                          # c_left = 0: fresh water enters
        R[0, j, 0] += F
        R[1, j, 0] += 2.0 * rho(c[j, 0]) * phi[j, 0] * Dm * (c[j, 0] - 0.0) / 1.0
        u = -(K[j, 2] / mu) * (pb[j] - p[j, 2]) / 0.5
        if u < 0:                                                       # seawater enters at rho1, c = 1
            branches.add(("right", "in"))
            R[0, j, 2] += 1025.0 * u
            R[1, j, 2] += 1025.0 * u * 1.0
        else:
            branches.add(("right", "out"))
            R[0, j, 2] += rho(c[j, 2]) * u
            R[1, j, 2] += rho(c[j, 2]) * u * c[j, 2]
    assert branches >= {("east", True), ("east", False), ("north", True), ("north", False),
                        ("right", "in"), ("right", "out")}
    d = H.Discretisation(pr, g, phi, K, u_in)
    Rp, Rc = d.residual(p.ravel(), c.ravel(), c_old.ravel())
    scale = np.abs(R).max()
    assert np.abs(Rp - R[0].ravel()).max() <= 1e-13 * scale
    assert np.abs(Rc - R[1].ravel()).max() <= 1e-13 * scale
