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


def _run(theta, nx, ny, nsteps, prob_kw, procs):
    from oracle import henry as H
    kw = dict(prob_kw or {})
    if "right_c_dirichlet" in kw:
        kw["right_c_dirichlet"] = bool(kw["right_c_dirichlet"])
    pr = H.Problem(**kw)
    g = H.Grid(nx, ny, nsteps)
    rs = H.solve_batch(pr, g, np.asarray(theta), processes=procs)
    return dict(c=np.stack([r.c.reshape(ny, nx) for r in rs]), p=np.stack([r.p.reshape(ny, nx) for r in rs]),
                qoi=np.array([r.qoi for r in rs]), its=np.array([r.newton_its for r in rs]),
                conv=np.array([r.converged for r in rs]),
                dsalt=np.array([r.max_salt_defect for r in rs]), dfluid=np.array([r.max_fluid_defect for r in rs]))


def oracle_batch(theta, nx, ny, nsteps, prob_kw=None, procs=NPROC):
    """dict of arrays c [S,ny,nx], p, qoi [S], its, conv, dsalt, dfluid."""
    with tempfile.TemporaryDirectory() as d:
        np.save(os.path.join(d, "theta.npy"), np.asarray(theta, dtype=np.float64))
        spec = dict(nx=nx, ny=ny, nsteps=nsteps, prob_kw=prob_kw or {}, procs=procs)
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
    out = _run(th, spec["nx"], spec["ny"], spec["nsteps"], spec["prob_kw"], spec["procs"])
    np.savez(os.path.join(d, "out.npz"), **out)
