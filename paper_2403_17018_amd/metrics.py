"""Run metrics as JSON lines: one object per solved batch (per level of a multilevel run).

A record holds the batch's grid and size; wall seconds and sample-timesteps/s when timed;
histograms over the samples of Newton iterations per time step and BiCGStab iterations per
Newton iteration; failures by status code; the worst fluid and salt mass-balance defects; and,
when the library's profiler ran, each kernel class's launches, milliseconds and, for the
bandwidth-bound classes, achieved GB/s and fraction of the 8 TB/s HBM peak.  Errors against
the CPU oracle belong to the tests, which run it; the product never does.

    with MetricsLog("run.jsonl") as log:
        r = hx.solve(theta, g)
        log.write(batch_record("level 3", g, r, seconds=dt, prof=hx.profile_read()))
"""
from __future__ import annotations

import json
import time

import numpy as np

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E

# Algorithmic bytes per unit of each bandwidth-bound kernel class (FP64 / FP32 multigrid): what
# one launch must move per cell-sample (per swept cell for the smoother, per fine cell for the
# restriction), counted from the arrays the kernel reads and writes.  The profiler's units are
# the cell-samples each launch covers.
BYTES_PER_UNIT = {
    64: dict(gs=208, spmv=136, assemble=216, restrict=76, prolong=216),
    32: dict(gs=104, spmv=96, assemble=136, restrict=38, prolong=108),
}
# The vertex-centred path (henry_vc_solve), per vertex-sample: the four-colour pass reads the
# 36-entry Jacobian row and b, writes x and reads the other three colours' x once (3 x 16 B
# per swept vertex); the SpMV reads J and x and writes y; the assembly reads p, c, c_old and
# one element's phi and K per vertex and writes R and J.
# With the FP32 multigrid the Jacobian and the cycle's vectors are FP32 (the SpMV's x and y stay
# FP64).
VC_BYTES_PER_UNIT = {
    64: dict(gs=288 + 16 + 16 + 48, spmv=288 + 16 + 16, assemble=16 + 8 + 16 + 16 + 288),
    32: dict(gs=144 + 8 + 8 + 24, spmv=144 + 16 + 16, assemble=16 + 8 + 16 + 16 + 144),
}


def _hist(x: np.ndarray, width: float) -> dict:
    """Fixed-width histogram of x (edges on multiples of width) with min, mean and max."""
    if x.size == 0:
        return dict(edges=[], counts=[], min=None, mean=None, max=None)
    lo = np.floor(x.min() / width) * width
    hi = np.floor(x.max() / width) * width + width
    edges = np.arange(lo, hi + 0.5 * width, width)
    counts, _ = np.histogram(x, edges)
    return dict(edges=[round(float(e), 6) for e in edges], counts=[int(c) for c in counts],
                min=float(x.min()), mean=float(x.mean()), max=float(x.max()))


def kernel_classes(prof: dict, mg_precision: int = 64) -> dict:
    """{class: {launches, units, ms[, avg_launch_us, gbs, frac_of_peak]}} from Henry.profile_read()."""
    out = {}
    table = BYTES_PER_UNIT[mg_precision]
    for name, (n, units, ms) in prof.items():
        if n == 0:
            continue
        row = dict(launches=int(n), units=int(units), ms=round(float(ms), 4))
        if name in table and ms > 0:
            gbs = units * table[name] / (ms * 1e-3) / 1e9
            row.update(avg_launch_us=round(ms / n * 1e3, 3), gbs=round(gbs, 2), frac_of_peak=round(gbs / HBM_PEAK_GBS, 4))
        out[name] = row
    return out


def batch_record(label: str, grid, result, seconds: float | None = None, prof: dict | None = None,
                 mg_precision: int = 64, **extra) -> dict:
    """One JSON-ready record for a SolveResult on henry_grid `grid`."""
    st = result.stats.detach().cpu().numpy().astype(np.float64)       # [S, 4] (or [S, 2])
    status = result.status.detach().cpu().numpy()
    S = st.shape[0]
    newton = st[:, 0]
    codes, counts = np.unique(status, return_counts=True)
    rec = dict(time=time.time(), label=label, nx=int(grid.nx), ny=int(grid.ny), nsteps=int(grid.nsteps),
               samples=int(S), mg_precision=int(mg_precision),
               newton_per_step=_hist(newton / max(grid.nsteps, 1), 0.25),
               krylov_per_newton=_hist(st[:, 1] / np.maximum(newton, 1.0), 0.25),
               failed=int(result.nfailed), status_counts={str(int(k)): int(v) for k, v in zip(codes, counts)},
               max_fluid_defect=float(st[:, 2].max()) if S and st.shape[1] > 3 else None,
               max_salt_defect=float(st[:, 3].max()) if S and st.shape[1] > 3 else None)
    if seconds is not None and seconds > 0:
        rec.update(seconds=float(seconds), sample_timesteps_per_s=S * grid.nsteps / seconds)
    if prof is not None:
        rec["kernel_classes"] = kernel_classes(prof, mg_precision)
    rec.update(extra)
    return rec


class MetricsLog:
    """Append-only JSON-lines file; each write() is one line, flushed at once."""

    def __init__(self, path: str):
        self.path = path
        self._f = open(path, "a", encoding="utf-8")

    def write(self, record: dict) -> None:
        self._f.write(json.dumps(record, separators=(",", ":")) + "\n")
        self._f.flush()

    def close(self) -> None:
        if not self._f.closed:
            self._f.close()

    def __enter__(self) -> "MetricsLog":
        return self

    def __exit__(self, *exc) -> None:
        self.close()
