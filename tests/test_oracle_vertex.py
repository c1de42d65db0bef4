"""Pins of the vertex-centred oracle (the paper's discretisation, section 2.3) against what
the paper and the mathematics fix, independently of the oracle's own code paths."""
import numpy as np
import pytest

from oracle import henry as H
from oracle import vertex as V

GOLDEN = "tests/golden/paper_table2.txt"


def _table2():
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    return [(int(r[0]), int(r[1]), int(r[2]), float(r[3])) for r in rows]


def test_hierarchy_matches_table2():
    """Table 2: vertex counts n_l, steps r_l and tau_l = 6016 / r_l of levels 0..3."""
    for level, n, r, tau in _table2():
        g = V.level_grid(level)
        assert V.vertex_count(g) == n
        assert g.nsteps == r
        assert 6016.0 / g.nsteps == tau
    # the text's coarse grid of 512 quadrilaterals with two unknowns per vertex: 1122
    assert 2 * V.vertex_count(H.Grid(32, 16, 1)) == 1122


def _disc(nx, ny, **kw):
    pr = H.Problem(**kw)
    g = H.Grid(nx, ny, 10)
    phi, K, u = H.sample_fields(pr, g, np.random.default_rng(0).normal(size=13) * 0.5)
    return pr, g, V.VCDiscretisation(pr, g, phi, K, u)


@pytest.mark.parametrize("c0", [0.0, 0.37, 1.0])
def test_hydrostatic_state_has_no_flux(c0):
    """Uniform c and p = p0 - rho(c) g y: the bilinear gradient is exact, so q = 0 on every
    box face and neither mass nor salt moves (whatever phi and K)."""
    pr, g, d = _disc(12, 6)
    c = np.full(d.nv, c0)
    p = 123.0 - H.rho(pr, c0) * pr.g * d.yv
    for f in d.faces(p, c):
        assert np.abs(f["F"]).max() <= 1e-12 * H.rho(pr, c0) * 1e-4
        assert np.abs(f["G"]).max() <= 1e-12 * H.rho(pr, c0) * 1e-4


def test_face_fluxes_cancel_between_boxes():
    """What leaves one box through a face enters the other: summed over all boxes, only the
    left-side inflow remains (fluid: rho(c_left) u_in Ly; salt: that times c_left)."""
    rng = np.random.default_rng(3)
    pr, g, d = _disc(10, 7, c_left=0.25)
    p = -pr.rho0 * pr.g * d.yv + rng.normal(size=d.nv) * 50.0
    c = rng.uniform(size=d.nv)
    Fp, Fc = d.flux_balance(p, c)
    qin = H.rho(pr, 0.25) * d.u_in_t * pr.Ly
    assert abs(Fp.sum() + qin) <= 1e-12 * np.abs(Fp).sum()
    assert abs(Fc.sum() + qin * 0.25) <= 1e-12 * np.abs(Fc).sum()


def test_upwind_fraction():
    F = np.array([0.0, 1.0, 2.0, 4.0, -4.0, 10.0])
    D = np.ones_like(F)
    assert np.array_equal(V.upwind_fraction(F, D), [0.0, 0.0, 0.0, 0.5, 0.5, 0.8])


def _steady_1d(nx, ny):
    """rho1 = rho0 and uniform fields: the flow is uniform (u_in along x) and the steady salt
    profile depends on x only; returns the oracle's steady state and the face Peclet number."""
    pr = H.Problem(rho1=1000.0, phi_amp=0.0, logK_amp=0.0, q_in_amp=0.0)
    g = H.Grid(nx, ny, 1)
    r = V.solve_sample(pr, g, np.zeros(13), tau=1e13, opts=H.SolveOptions(newton_tol=1e-13, newton_maxit=50))
    assert r.converged
    hx = pr.Lx / nx
    pe = pr.q_in * hx / (pr.phi_mean * pr.Dm)
    return pr, r, pe


@pytest.mark.parametrize("nx,ny", [(16, 8), (32, 16)])
def test_steady_1d_central_regime_is_the_exact_discrete_solution(nx, ny):
    """Face Peclet number Pe = u hx / (phi D_m) < 2: every face is central, and the steady
    discrete equations are the three-point recursion (D + F/2) c_{i-1} - 2 D c_i + (D - F/2) c_{i+1} = 0
    with c_0 = 0, c_nx = 1, whose solution is c_i = (r^i - 1) / (r^nx - 1), r = (1 + Pe/2) / (1 - Pe/2)."""
    pr, r, pe = _steady_1d(nx, ny)
    assert pe < 2.0
    ratio = (1.0 + pe / 2.0) / (1.0 - pe / 2.0)
    i = np.arange(nx + 1)
    exact = (ratio ** i - 1.0) / (ratio ** nx - 1.0)
    c = r.c.reshape(ny + 1, nx + 1)
    assert np.abs(c - exact[None, :]).max() <= 1e-10


def test_steady_1d_upwind_regime_keeps_the_inflow_value():
    """Pe > 2: the upwind fraction w = 1 - 2/Pe removes the downstream coupling exactly, so the
    steady interior holds the inflow value c_left = 0 up to the Dirichlet column c = 1."""
    pr, r, pe = _steady_1d(8, 4)
    assert pe > 2.0
    c = r.c.reshape(5, 9)
    assert np.abs(c[:, :-1]).max() <= 1e-12
    assert np.all(c[:, -1] == 1.0)


def test_coloured_jacobian_equals_plain_differences():
    """The coloured central differences agree with one column at a time."""
    rng = np.random.default_rng(5)
    pr, g, d = _disc(4, 3)
    p = -pr.rho0 * pr.g * d.yv + rng.normal(size=d.nv) * 20.0
    c = rng.uniform(0.1, 0.9, size=d.nv)
    c_old = rng.uniform(0.1, 0.9, size=d.nv)
    Jc = d.jacobian_fd(p, c, c_old).toarray()
    u = np.empty(2 * d.nv); u[0::2], u[1::2] = p, c
    Jp = np.zeros_like(Jc)
    for k in range(2 * d.nv):
        e = np.zeros_like(u)
        e[k] = pr.rho0 * pr.g * pr.Ly * 1e-7 if k % 2 == 0 else 1e-5
        Jp[:, k] = (d.residual_vector(u + e, c_old) - d.residual_vector(u - e, c_old)) / (2.0 * e[k])
    assert np.abs(Jc - Jp).max() <= 1e-12 * np.abs(Jp).max()


def test_qoi_hand_values():
    """Q = sum c rho(c) |box n {x > 1}|: c = 1 gives rho1 * 1 m^2, c = 1/2 gives 0.5 (rho0 + rho1)/2."""
    pr = H.Problem()
    for g in (H.Grid(16, 8, 1), H.Grid(9, 4, 1)):    # x = 1 on a vertex, and between vertices
        nv = V.vertex_count(g)
        assert V.qoi_salt_mass(pr, g, np.ones(nv)) == pytest.approx(1025.0, rel=1e-14)
        assert V.qoi_salt_mass(pr, g, np.full(nv, 0.5)) == pytest.approx(0.5 * 1012.5, rel=1e-14)
        c = np.zeros(nv).reshape(g.ny + 1, g.nx + 1)
        c[:, : g.nx // 2 - 1] = 1.0                  # salt only at x < 1: nothing counts
        assert V.qoi_salt_mass(pr, g, c.ravel()) == 0.0


def test_mass_balance_over_steps():
    """Storage change plus the flux through the boundary and into the Dirichlet vertices
    balances to the Newton tolerance in every step (fluid and salt)."""
    pr = H.Problem()
    r = V.solve_sample(pr, V.level_grid(0), np.random.default_rng(7).normal(size=13), nsteps=12)
    assert r.converged
    assert r.max_fluid_defect <= 1e-9 and r.max_salt_defect <= 1e-9
    assert 0.0 <= r.c.min() and r.c.max() <= 1.0 + 1e-9


def test_box_volumes_add_up_to_the_pore_volume():
    pr, g, d = _disc(7, 5)
    assert d.box.sum() == pytest.approx(d.phi.sum() * d.hx * d.hy, rel=1e-14)
    # an interior vertex owns a quarter of each of its four elements
    phi = d.phi.reshape(5, 7)
    assert d.box[d.vid[2, 3]] == pytest.approx(0.25 * d.hx * d.hy * phi[1:3, 2:4].sum(), rel=1e-14)


def test_face_fluxes_at_their_integration_points():
    """p = a x y + p0 and c = b x + e (y + Ly) are reproduced exactly by the bilinear
    interpolation, so each face's flux is the closed form at its own integration point:
    x-faces at (x_i + hx/2, y_j + hy/4 or 3hy/4), y-faces at (x_i + 3hx/4 or hx/4, y_j + hy/2),
    with rho taken at that point (not at the face's two vertices)."""
    pr, g, d = _disc(6, 4)
    a, p0, b, e = 300.0, 50.0, 0.15, 0.1
    p = a * d.xv * d.yv + p0
    c = b * d.xv + e * (d.yv + pr.Ly)
    faces = d.faces(p, c)
    ei, ej = np.meshgrid(np.arange(6), np.arange(4))
    xi, yj = (ei * d.hx).ravel(), (-pr.Ly + ej * d.hy).ravel()
    K = d.K
    for k, (s, t, axis) in enumerate(((0.5, 0.25, 0), (0.75, 0.5, 1), (0.5, 0.75, 0), (0.25, 0.5, 1))):
        x, y = xi + s * d.hx, yj + t * d.hy
        r = H.rho(pr, b * x + e * (y + pr.Ly))
        if axis == 0:
            F = r * (-(K / pr.mu) * a * y) * 0.5 * d.hy
            Gd = r * d.phi * pr.Dm * b * 0.5 * d.hy
        else:
            F = r * (-(K / pr.mu) * (a * x + r * pr.g)) * 0.5 * d.hx
            Gd = r * d.phi * pr.Dm * e * 0.5 * d.hx
        assert np.abs(faces[k]["F"] - F).max() <= 1e-12 * np.abs(F).max(), k
        # G = F c_conv - diffusive part: the diffusive part is exact at the same point
        ca, cb = c[faces[k]["a"]], c[faces[k]["b"]]
        w = faces[k]["w"]
        conv = faces[k]["F"] * ((1 - w) * 0.5 * (ca + cb) + w * np.where(faces[k]["F"] >= 0, ca, cb))
        assert np.abs((conv - faces[k]["G"]) - Gd).max() <= 1e-12 * np.abs(Gd).max(), k


def test_steady_seawater_column_is_hydrostatic():
    """c = 1 on both sides and no inflow: the steady state is a resting column of seawater, so
    c = 1 everywhere and p = -rho1 g y (zero at the top, the right side's hydrostatic datum)."""
    pr = H.Problem(q_in=0.0, c_left=1.0)
    g = H.Grid(8, 4, 1)
    # one implicit step long enough that the storage term no longer moves the state (the mass
    # balance defects, relative to the inflow, are undefined without inflow)
    with np.errstate(divide="ignore", invalid="ignore"):
        r = V.solve_sample(pr, g, np.zeros(13), tau=1e17, opts=H.SolveOptions(newton_tol=1e-13, newton_maxit=60))
    assert r.converged
    yv = np.repeat(-pr.Ly + np.arange(5) * pr.Ly / 4, 9)
    assert np.abs(r.c - 1.0).max() <= 1e-10
    assert np.abs(r.p - (-pr.rho1 * pr.g * yv)).max() <= 1e-9 * pr.rho1 * pr.g * pr.Ly
