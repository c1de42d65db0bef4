"""Karhunen-Loeve eigenpairs of the separable exponential covariance (oracle).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper models porosity by L2-orthogonal sin/cos functions that mimic a KL
expansion (section 4, "Uncertain porosity and recharge"); the workload studied
here uses a true KL expansion with exponential covariance, correlation length
b = 0.5 m and unit variance:

    C(x, x') = exp(-|x1 - x1'| / b) * exp(-|x2 - x2'| / b)   on [0,2] x [-1,0].

The kernel is a product, so the 2-D eigenpairs are products of 1-D ones.  On an
interval of half-length a centred at s_c the 1-D integral equation
    int exp(-|s - t| / b) f(t) dt = lam f(s)
has the classical closed form (Ghanem & Spanos 1991, section 2.3), c = 1/b:
  even modes  f = cos(w (s - s_c)),  w tan(w a) = c
  odd modes   f = sin(w (s - s_c)),  w + c tan(w a) = 0
with lam = 2 c / (w^2 + c^2).  Normalised in L2 over the interval.  The 2-D
modes are sorted by eigenvalue, descending (ties: smaller x-index first).
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import brentq


def roots_1d(a: float, b: float, nmodes: int):
    """First ``nmodes`` 1-D modes, sorted by decreasing eigenvalue.

    Returns list of (omega, parity, lam, norm) with parity 0 = even (cos), 1 = odd (sin)
    and norm = sqrt(int_{-a}^{a} f^2).
    """
    c = 1.0 / b
    out = []
    k = 0
    while len(out) < nmodes:
        # even root in (k pi / a, (k + 1/2) pi / a)
        lo, hi = k * np.pi / a, (k + 0.5) * np.pi / a
        eps = 1e-14 * hi + 1e-300
        w = brentq(lambda w: w * np.tan(w * a) - c, lo + eps, hi - eps, xtol=1e-15, rtol=1e-15, maxiter=500)
        out.append((w, 0))
        # odd root in ((k + 1/2) pi / a, (k + 1) pi / a)
        lo, hi = (k + 0.5) * np.pi / a, (k + 1) * np.pi / a
        eps = 1e-14 * hi
        w = brentq(lambda w: w + c * np.tan(w * a), lo + eps, hi - eps, xtol=1e-15, rtol=1e-15, maxiter=500)
        out.append((w, 1))
        k += 1
    res = []
    for w, par in out:
        lam = 2.0 * c / (w * w + c * c)
        if par == 0:
            nrm2 = a + np.sin(2.0 * w * a) / (2.0 * w)
        else:
            nrm2 = a - np.sin(2.0 * w * a) / (2.0 * w)
        res.append((w, par, lam, np.sqrt(nrm2)))
    res.sort(key=lambda t: -t[2])   # omegas increase => lam decreases; keeps order
    return res[:nmodes]


def eval_1d(mode, s, s_c):
    w, par, _, nrm = mode
    t = np.asarray(s, dtype=np.float64) - s_c
    return (np.cos(w * t) if par == 0 else np.sin(w * t)) / nrm


class KL2D:
    """Separable 2-D KL basis on [0, Lx] x [-Ly, 0]."""

    def __init__(self, Lx=2.0, Ly=1.0, corr_len=0.5, nmodes=8, n1d=12):
        self.Lx, self.Ly, self.b = Lx, Ly, corr_len
        self.mx = roots_1d(Lx / 2, corr_len, n1d)
        self.my = roots_1d(Ly / 2, corr_len, n1d)
        pairs = []
        for ix, mx in enumerate(self.mx):
            for iy, my in enumerate(self.my):
                pairs.append((mx[2] * my[2], ix, iy))
        pairs.sort(key=lambda t: (-t[0], t[1]))
        self.pairs = pairs[:nmodes]
        self.lam = np.array([p[0] for p in self.pairs])

    def eval(self, k, x, y):
        _, ix, iy = self.pairs[k]
        return eval_1d(self.mx[ix], x, self.Lx / 2) * eval_1d(self.my[iy], y, -self.Ly / 2)

    def table(self, x, y):
        """E[k, ...] = e_k(x, y) for all modes k."""
        return np.stack([self.eval(k, x, y) for k in range(len(self.pairs))])
