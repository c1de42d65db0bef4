"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

This module holds no arithmetic of the method itself: it only draws the
random parameter vectors theta and names the workload shapes.  Both the
oracle and the HIP library receive the same theta array, so neither side
needs its own random number generator.

Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC'11), a counter-based generator.  One call per
(level, sample, component) with key = (seed, 0) and counter =
(level, sample, component, 0).  Uniforms take 53 bits from two 32-bit words;
normals use the Box-Muller transform of two such uniforms (cosine branch only).

theta layout per sample (13 values, row-major ``theta[s, k]``):
  k = 0..3   xi_k   ~ U[-1, 1]   porosity KL coefficients
  k = 4..11  eta_k  ~ N(0, 1)    log-permeability KL coefficients
  k = 12     zeta   ~ U[-1, 1]   recharge factor
The paper's own model (section 4) reads xi_1 = theta[0], xi_2 = theta[1] and
xi_3 = theta[12] of the same layout; qmc_theta() fills those from the Halton
sequence for its quasi-Monte Carlo runs (section 5, 600 points).
"""
from __future__ import annotations

import numpy as np

N_THETA = 13
N_XI = 4
N_ETA = 8
IDX_XI = slice(0, 4)
IDX_ETA = slice(4, 12)
IDX_ZETA = 12

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint64(0x9E3779B9)
_W1 = np.uint64(0xBB67AE85)
_MASK32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(counter, key):
    """Philox4x32 with 10 rounds, vectorised over leading axes.

    counter: uint array [..., 4]; key: uint array [..., 2].  Returns uint32 [..., 4].
    """
    c = np.asarray(counter, dtype=np.uint64) & _MASK32
    k = np.asarray(key, dtype=np.uint64) & _MASK32
    c0, c1, c2, c3 = (c[..., i].copy() for i in range(4))
    k0, k1 = k[..., 0].copy(), k[..., 1].copy()
    for rnd in range(10):
        p0 = _M0 * c0            # fits in 64 bits: 32x32 -> 64
        p1 = _M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0) & _MASK32, lo1, (hi0 ^ c3 ^ k1) & _MASK32, lo0
        if rnd < 9:
            k0 = (k0 + _W0) & _MASK32
            k1 = (k1 + _W1) & _MASK32
    return np.stack([c0, c1, c2, c3], axis=-1).astype(np.uint32)


def _u53(hi, lo):
    """Two 32-bit words -> uniform in (0, 1] with 53 random bits."""
    hi = hi.astype(np.uint64) >> np.uint64(6)   # 26 bits
    lo = lo.astype(np.uint64) >> np.uint64(5)   # 27 bits
    m = (hi << np.uint64(27)) | lo              # 53 bits
    return (m.astype(np.float64) + 1.0) * (1.0 / 9007199254740992.0)


def draw_theta(seed: int, nsamples: int, level: int = 0, first_sample: int = 0) -> np.ndarray:
    """theta[nsamples, 13] for one MLMC level, float64.

    A coarse partner of level ``level`` reuses exactly this array (coupled pair).
    """
    s = np.arange(first_sample, first_sample + nsamples, dtype=np.uint64)
    comp = np.arange(N_THETA, dtype=np.uint64)
    S, Cc = np.meshgrid(s, comp, indexing="ij")
    ctr = np.stack([np.full_like(S, level), S, Cc, np.zeros_like(S)], axis=-1)
    key = np.zeros(ctr.shape[:-1] + (2,), dtype=np.uint64)
    key[..., 0] = np.uint64(seed)
    w = philox4x32_10(ctr, key)
    u1 = _u53(w[..., 0], w[..., 1])
    u2 = _u53(w[..., 2], w[..., 3])
    th = 2.0 * u1 - 1.0
    normal = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
    th[:, IDX_ETA] = normal[:, IDX_ETA]
    return np.ascontiguousarray(th)


def halton(n: int, bases=(2, 3, 5), start: int = 1) -> np.ndarray:
    """Points start..start+n-1 of the Halton sequence, [n, len(bases)] in [0, 1).

    Coordinate d of point i is the radical inverse of i in base bases[d]: the base-b
    digits of i mirrored about the radix point.  Unscrambled; start = 1 skips the origin.
    """
    idx = np.arange(start, start + n, dtype=np.int64)
    out = np.zeros((n, len(bases)))
    for d, b in enumerate(bases):
        i = idx.copy()
        f = 1.0 / b
        while (i > 0).any():
            out[:, d] += f * (i % b)
            i //= b
            f /= b
    return out


def qmc_theta(n: int, start: int = 1) -> np.ndarray:
    """theta[n, 13] for the paper's own model (section 4) from the Halton sequence in bases
    2, 3, 5: xi_1 = theta[0], xi_2 = theta[1], xi_3 = theta[12], each 2u - 1 in [-1, 1);
    the other components are 0 (unused by that model)."""
    u = halton(n, (2, 3, 5), start)
    th = np.zeros((n, N_THETA))
    th[:, 0] = 2.0 * u[:, 0] - 1.0
    th[:, 1] = 2.0 * u[:, 1] - 1.0
    th[:, IDX_ZETA] = 2.0 * u[:, 2] - 1.0
    return th


def level_grid(level: int):
    """(nx, ny, nsteps) of MLMC level l: 32*2^l x 16*2^l cells, 48*2^l steps."""
    return 32 << level, 16 << level, 48 << level


# Workloads: shapes, sample counts and seeds of the five configurations.
WORKLOADS = {
    "c1_fp64_level0": dict(level=0, nsamples=16, seed=0, mg_precision=64),
    "c2_fp64_level3": dict(level=3, nsamples=512, seed=1, mg_precision=64),
    "c3_mixed_level4": dict(level=4, nsamples=128, seed=2, mg_precision=32),
    "c4_mlmc_levels0to4": dict(levels=(0, 1, 2, 3, 4), nsamples=(4096, 1024, 256, 64, 16), seed=3),
    "c5_adjoint_level3": dict(level=3, nsamples=256, seed=4, checkpoint_every=32),
}
