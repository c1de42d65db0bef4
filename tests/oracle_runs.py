"""Run the CPU oracle on the same seeded inputs as the GPU path (tests only).

oracle_batch() runs the oracle in a fresh child interpreter, so a test process that
has initialised the GPU never forks; the child fans the samples out over a process pool.
"""
import json
import os
import subprocess
import sys
import tempfile

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NPROC = min(16, os.cpu_count() or 1)


FW_BAND = 1e-8   # |c - threshold| below which the fresh-water indicator may differ between solvers


def _series_one(args):
    """Per-step series of one sample plus, per step, the area of the cells whose c lies
    within FW_BAND of the fresh-water threshold (where the indicator is not decided)."""
    from oracle import henry as H
    pr, g, th = args
    r = H.solve_sample(pr, g, th, keep_states=True, series=True)
    hx, hy = g.h(pr)
    amb = np.array([np.count_nonzero(np.abs(c - H.FW_THRESHOLD) <= FW_BAND) * hx * hy for _, c in r.states[1:]])
    return r, amb


def _run(theta, nx, ny, nsteps, prob_kw, procs, series=False):
    from oracle import henry as H
    kw = dict(prob_kw or {})
    if "right_c_dirichlet" in kw:
        kw["right_c_dirichlet"] = bool(kw["right_c_dirichlet"])
    pr = H.Problem(**kw)
    g = H.Grid(nx, ny, nsteps)
    extra = {}
    if series:
        import multiprocessing as mp
        jobs = [(pr, g, t) for t in np.asarray(theta)]
        with mp.get_context("fork").Pool(procs) as pool:
            out = pool.map(_series_one, jobs)
        rs = [r for r, _ in out]
        extra = dict(series=np.stack([r.series for r in rs]), fw_ambiguous=np.stack([a for _, a in out]))
        for r in rs:
            r.states = None
    else:
        rs = H.solve_batch(pr, g, np.asarray(theta), processes=procs)
    return dict(c=np.stack([r.c.reshape(ny, nx) for r in rs]), p=np.stack([r.p.reshape(ny, nx) for r in rs]),
                qoi=np.array([r.qoi for r in rs]), its=np.array([r.newton_its for r in rs]),
                conv=np.array([r.converged for r in rs]),
                dsalt=np.array([r.max_salt_defect for r in rs]), dfluid=np.array([r.max_fluid_defect for r in rs]),
                **extra)


def _vc_one(args):
    from oracle import vertex as V
    pr, g, th = args
    return V.solve_sample(pr, g, th)


def _run_vertex(theta, nx, ny, nsteps, prob_kw, procs):
    import multiprocessing as mp
    from oracle import henry as H
    pr = H.Problem(**(prob_kw or {}))
    g = H.Grid(nx, ny, nsteps)
    jobs = [(pr, g, t) for t in np.asarray(theta)]
    with mp.get_context("fork").Pool(max(1, min(procs, len(jobs)))) as pool:
        rs = pool.map(_vc_one, jobs)
    return dict(c=np.stack([r.c.reshape(ny + 1, nx + 1) for r in rs]), p=np.stack([r.p.reshape(ny + 1, nx + 1) for r in rs]),
                qoi=np.array([r.qoi for r in rs]), its=np.array([r.newton_its for r in rs]),
                conv=np.array([r.converged for r in rs]),
                dsalt=np.array([r.max_salt_defect for r in rs]), dfluid=np.array([r.max_fluid_defect for r in rs]))


def vc_oracle_batch(theta, nx, ny, nsteps, prob_kw=None, procs=NPROC):
    """The vertex-centred oracle (oracle.vertex) on nx x ny elements: c, p [S, ny+1, nx+1], qoi,
    its, conv, dsalt, dfluid [S]."""
    with tempfile.TemporaryDirectory() as d:
        np.save(os.path.join(d, "theta.npy"), np.asarray(theta, dtype=np.float64))
        spec = dict(nx=nx, ny=ny, nsteps=nsteps, prob_kw=prob_kw or {}, procs=procs, scheme="vertex")
        with open(os.path.join(d, "spec.json"), "w") as f:
            json.dump(spec, f)
        env = dict(os.environ, PYTHONPATH=ROOT + os.pathsep + os.environ.get("PYTHONPATH", ""))
        subprocess.run([sys.executable, "-m", "tests.oracle_runs", d], check=True, cwd=ROOT, env=env)
        z = np.load(os.path.join(d, "out.npz"))
        return {k: z[k] for k in z.files}


def oracle_batch(theta, nx, ny, nsteps, prob_kw=None, procs=NPROC, series=False):
    """dict of arrays c [S,ny,nx], p, qoi [S], its, conv, dsalt, dfluid; with series=True
    also series [S, nsteps, 17] and fw_ambiguous [S, nsteps] (see _series_one)."""
    with tempfile.TemporaryDirectory() as d:
        np.save(os.path.join(d, "theta.npy"), np.asarray(theta, dtype=np.float64))
        spec = dict(nx=nx, ny=ny, nsteps=nsteps, prob_kw=prob_kw or {}, procs=procs, series=series)
        with open(os.path.join(d, "spec.json"), "w") as f:
            json.dump(spec, f)
        env = dict(os.environ, PYTHONPATH=ROOT + os.pathsep + os.environ.get("PYTHONPATH", ""))
        subprocess.run([sys.executable, "-m", "tests.oracle_runs", d], check=True, cwd=ROOT, env=env)
        z = np.load(os.path.join(d, "out.npz"))
        return {k: z[k] for k in z.files}


def defect_bound(theta, prob, nx, ny, nsteps, newton_tol=1e-9, u_max=1e-2):
    """Largest per-step mass-balance defect an accepted Newton iterate can show, per sample:
    (fluid bound [S], salt bound [S]), in the GPU's unit (storage change + tau * boundary
    outflux, over one step's inflow tau rho0 u_in Ly).

    Derivation (first order in the tolerance).  Interior fluxes cancel, so the defect of an
    iterate u is tau |sum_P R_P(u)| / scale, and sum_P R_P is the total storage change plus the
    boundary outflux.  The accepted iterate lies within one Newton update of the step's discrete
    solution u*, where sum_P R_P(u*) = 0; the stopping test (or, for the predictive stop, the
    predicted update) bounds that update by |dc| <= tol and |dp| <= tol rho0 g Ly.  To first
    order the defect is then at most the sum over cells of |d(storage + boundary outflux)/du|
    times those bounds, with c in [0, 1]:
      storage    fluid vol phi drho / tau,  salt vol phi (rho0 + 2 drho) / tau  (per |dc|);
      left face  salt 2 phi Dm (drho + rho1) hy/hx                            (per |dc|);
      right face d F/d p = 2 rho1 K / mu (times |dp|; also in the salt flux, c_b <= 1) and
                 d F/d c = drho |u| hy, d G/d c <= (drho + rho1) |u| hy with |u| <= u_max
                 (times |dc|); the Dirichlet variant adds 2 phi Dm (drho + rho1) hy/hx.
    prob: the oracle's Problem (fields and constants); theta [S, 13]."""
    from oracle import henry as H
    g = H.Grid(nx, ny, nsteps)
    hx, hy = g.h(prob)
    tau = prob.T / nsteps
    dr = prob.rho1 - prob.rho0
    dc = newton_tol
    dp = newton_tol * prob.rho0 * prob.g * prob.Ly
    vol = hx * hy
    bf, bs = [], []
    for th in np.asarray(theta):
        phi, K, u_in = H.sample_fields(prob, g, th)
        Kr, phr, phl = K[:, -1], phi[:, -1], phi[:, 0]
        dFdp = 2.0 * prob.rho1 * Kr / prob.mu
        fluid = vol * phi.sum() * dr / tau * dc + (dFdp * dp + dr * u_max * hy * dc).sum()
        salt = vol * phi.sum() * (prob.rho0 + 2.0 * dr) / tau * dc
        salt += (2.0 * phl * prob.Dm * (dr + prob.rho1) * hy / hx).sum() * dc
        salt += (dFdp * dp + (2.0 * dr + prob.rho1) * u_max * hy * dc).sum()
        if prob.right_c_dirichlet:
            salt += (2.0 * phr * prob.Dm * (dr + prob.rho1) * hy / hx).sum() * dc
        scale = prob.rho0 * u_in * prob.Ly
        bf.append(fluid / scale)
        bs.append(salt / scale)
    return np.array(bf), np.array(bs)


def rel_inf(a, b):
    """Per-sample normwise relative error max|a-b| / max|b| over the leading sample axis."""
    a = np.asarray(a).reshape(a.shape[0], -1)
    b = np.asarray(b).reshape(b.shape[0], -1)
    return np.abs(a - b).max(axis=1) / np.abs(b).max(axis=1)


if __name__ == "__main__":
    d = sys.argv[1]
    spec = json.load(open(os.path.join(d, "spec.json")))
    th = np.load(os.path.join(d, "theta.npy"))
    if spec.get("scheme") == "vertex":
        out = _run_vertex(th, spec["nx"], spec["ny"], spec["nsteps"], spec["prob_kw"], spec["procs"])
    else:
        out = _run(th, spec["nx"], spec["ny"], spec["nsteps"], spec["prob_kw"], spec["procs"], spec.get("series", False))
    np.savez(os.path.join(d, "out.npz"), **out)
