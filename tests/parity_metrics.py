"""Error measures shared by the GPU parity tests (test infrastructure).

relerr: ||a - b||_2 / ||b||_2 over all components (the per-evaluation
velocity error of one system, and the centre-displacement drift).

sphere_err: max over spheres of ||a_i - b_i||_2 / (||b_i||_2 + median_j
||b_j||_2): every sphere's error relative to its own speed, with the median
speed as the floor for slow spheres. The norm over a whole system dilutes a
wrong block of targets by about sqrt(N / block); this bounds every sphere,
so one wrong sphere shows at full size. (Relative to the median alone, a
sphere next to a steric contact, whose force is 10^3-10^4 times the typical
spring force, carries FP32 rounding of a term far larger than the median
speed.)
"""
from __future__ import annotations

import numpy as np

# AD_FP32C bars. Velocity: 1e-6 relative per evaluation over a system; drift:
# 1e-4 relative over the run.
NORM_BAR = 1e-6
DRIFT_BAR = 1e-4
# Per sphere: FP32 pair terms carry relative rounding of a few 2^-24 each and
# single-float positions of |x| <= 400 are rounded to 2^-16 (1.5e-5 absolute),
# which moves the term of a close neighbour (r ~ 2) by up to about 1e-5 of
# itself, and a neighbour's term is at most comparable to the sphere's own
# velocity. 2e-5 leaves room for that worst case and still fails any wrong
# index, sign or dropped term (those are O(1)).
SPHERE_BAR = 2e-5


def relerr(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def sphere_err(a, b, extra=None) -> float:
    """extra: an optional per-sphere addition to the scale (see
    near_term_scale)."""
    a = np.asarray(a, dtype=np.float64).reshape(-1, 3)
    b = np.asarray(b, dtype=np.float64).reshape(-1, 3)
    nb = np.linalg.norm(b, axis=1)
    scale = nb + np.median(nb)
    if extra is not None:
        scale = scale + np.asarray(extra, dtype=np.float64)
    return float((np.linalg.norm(a - b, axis=1) / scale).max())


def near_term_scale(X, F, eta=1.0, radius=8.0):
    """Per sphere, the sum of the magnitudes of the Oseen terms of its
    neighbours closer than `radius`, 2 |F_j| / (8 pi eta r_ij) each (the
    largest the term can be): the size of the terms whose FP32 rounding
    survives when they cancel each other, as around a steric contact, where
    the two forces are large, equal and opposite."""
    from scipy.spatial import cKDTree
    X = np.asarray(X, dtype=np.float64)
    Fn = np.linalg.norm(np.asarray(F, dtype=np.float64), axis=1)
    pairs = np.array(sorted(cKDTree(X).query_pairs(radius)), dtype=np.int64).reshape(-1, 2)
    out = np.zeros(X.shape[0])
    if len(pairs):
        i, j = pairs[:, 0], pairs[:, 1]
        r = np.linalg.norm(X[i] - X[j], axis=1)
        c = 2.0 / (8.0 * np.pi * eta * r)
        np.add.at(out, i, c * Fn[j])
        np.add.at(out, j, c * Fn[i])
    return out


def check_fp32c(a, b, what: str = "", norm_bar: float = NORM_BAR, sphere_bar: float = SPHERE_BAR, extra=None):
    """Both bars at once; returns (norm error, per-sphere error)."""
    e, s = relerr(a, b), sphere_err(a, b, extra)
    print(f"  {what} rel err {e:.2e}, per-sphere {s:.2e}", flush=True)
    assert e <= norm_bar, (what, e)
    assert s <= sphere_bar, (what, s)
    return e, s
