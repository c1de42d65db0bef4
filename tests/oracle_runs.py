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


def defect_bound(theta, tau, phi_max, q_in_amp=0.1, q_in=6.6e-5, newton_tol=1e-9, margin=5.0):
    """Largest per-step mass-balance defect allowed for accepted Newton iterates, per sample.

    The GPU reports the defect (storage change + tau * boundary outflux) of each step over
    one step's inflow tau rho0 u_in Ly.  The exact discrete fixed point balances to rounding;
    an iterate accepted at Newton tolerance tol may be off by about tol in c in every cell,
    which moves at most phi_max rho1 |Omega| tol of salt (and rho1 - rho0 times that of
    fluid).  `margin` covers the predictive stop, whose accepted iterate is only predicted
    to be within tol.  Returns the bound for every sample of theta [S, 13] (u_in from zeta).
    """
    u_in = q_in * (1.0 + q_in_amp * np.asarray(theta)[:, 12])
    return margin * phi_max * 1025.0 * 2.0 * newton_tol / (tau * 1000.0 * u_in * 1.0)


def rel_inf(a, b):
    """Per-sample normwise relative error max|a-b| / max|b| over the leading sample axis."""
    a = np.asarray(a).reshape(a.shape[0], -1)
    b = np.asarray(b).reshape(b.shape[0], -1)
    return np.abs(a - b).max(axis=1) / np.abs(b).max(axis=1)


if __name__ == "__main__":
    d = sys.argv[1]
    spec = json.load(open(os.path.join(d, "spec.json")))
    th = np.load(os.path.join(d, "theta.npy"))
    out = _run(th, spec["nx"], spec["ny"], spec["nsteps"], spec["prob_kw"], spec["procs"], spec.get("series", False))
    np.savez(os.path.join(d, "out.npz"), **out)
