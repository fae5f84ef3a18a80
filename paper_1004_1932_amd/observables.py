"""Observables of the pair and array experiments (Sec. IV), computed on the
host from recorded states: dumbbell centres (what `Simulator.run` records),
sphere positions (`Simulator.get_state`) or the stroke-averaged state.

These are analysis of the simulation's output, not part of the time step.
Systems are concatenated as everywhere else; S_per_sys gives their sizes.
"""
from __future__ import annotations

import numpy as np


def _np(a) -> np.ndarray:
    if hasattr(a, "detach"):
        a = a.detach().cpu().numpy()
    return np.asarray(a, dtype=np.float64)


def centres(X) -> np.ndarray:
    """Geometric centres R = (X_2s + X_2s+1) / 2, shape (S, 3)."""
    X = _np(X)
    return 0.5 * (X[0::2] + X[1::2])


def axes(X) -> np.ndarray:
    """Unit axes N = (X_2s+1 - X_2s) / |X_2s+1 - X_2s|, shape (S, 3)."""
    X = _np(X)
    n = X[1::2] - X[0::2]
    return n / np.linalg.norm(n, axis=1, keepdims=True)


def _segments(S_total: int, S_per_sys) -> np.ndarray:
    if S_per_sys is None:
        return np.array([0, S_total])
    off = np.zeros(len(S_per_sys) + 1, dtype=np.int64)
    off[1:] = np.cumsum(np.asarray(S_per_sys, dtype=np.int64))
    if off[-1] != S_total:
        raise ValueError(f"S_per_sys sums to {off[-1]}, the arrays hold {S_total} dumbbells")
    return off


def msd_per_system(R1, R0, S_per_sys=None) -> np.ndarray:
    """(1/S_b) sum over the dumbbells of system b of |R(t) - R(0)|^2: the
    inner average of the mean square displacement per particle (Sec. IV.C)."""
    R1, R0 = _np(R1), _np(R0)
    d2 = ((R1 - R0) ** 2).sum(1)
    off = _segments(len(d2), S_per_sys)
    return np.array([d2[off[b]:off[b + 1]].mean() for b in range(len(off) - 1)])


def ensemble_msd(R1, R0, S_per_sys=None) -> float:
    """<<R(t)^2>>: the per-system mean square displacement averaged over the
    W runs (systems) of an ensemble (Sec. IV.C)."""
    return float(msd_per_system(R1, R0, S_per_sys).mean())


def _pairs(A) -> np.ndarray:
    A = _np(A)
    if A.shape[0] % 2:
        raise ValueError("pair observables need two dumbbells per system")
    return A.reshape(-1, 2, 3)


def pair_mean_displacement(R1, R0) -> np.ndarray:
    """{[R^2(t) + R^1(t)] - [R^2(0) + R^1(0)]} / 2 for each two-dumbbell
    system, shape (n, 3) (Sec. IV.A)."""
    a, b = _pairs(R1), _pairs(R0)
    return 0.5 * ((a[:, 1] + a[:, 0]) - (b[:, 1] + b[:, 0]))


def pair_separation_change(R1, R0) -> np.ndarray:
    """[R^2(t) - R^1(t)] - [R^2(0) - R^1(0)] for each two-dumbbell system,
    shape (n, 3) (Sec. IV.A)."""
    a, b = _pairs(R1), _pairs(R0)
    return (a[:, 1] - a[:, 0]) - (b[:, 1] - b[:, 0])


def pair_projection(Nax) -> np.ndarray:
    """q = N^sigma . N^rho for each two-dumbbell system, shape (n,)
    (Sec. IV.B; Delta q(t) = q(t) - q(0))."""
    n = _pairs(Nax)
    return (n[:, 0] * n[:, 1]).sum(1)
