"""Initial conditions of the paper's pair and array experiments (Sec. IV).

* Parameters: the values printed for the aligned-pair experiment (Fig. 1
  caption) in SI units: ell = 5 um, omega = 500 /s (T = 2 pi / omega),
  lam = 0.1 ell, a = 0.2 ell, k_0 = 1e-3 kg/s^2, viscosity 1e-3 kg/(m s),
  time step about 1e-4 T. The pair and array experiments use the same model
  parameters (Sec. IV.B, IV.C).
* Rotating pairs (Sec. IV.B): dumbbell sigma at the origin along x, dumbbell
  rho at distance 5 ell on a circle in the x-y plane at angle theta, its axis
  in the plane with projection q(0) = N^sigma . N^rho held fixed as theta
  varies. The paper does not state the phases of this experiment; the
  phase difference of the aligned-pair experiment, pi/2, is used.
* Arrays (Sec. IV.C): centres on a cubic x-by-x-by-x lattice of spacing
  rho^(-1/3), centred at the origin; axes uniform on the unit sphere
  (normalised standard normal 3-vectors); phases either "checkerboard"
  (0 or pi/2, every nearest neighbour holding the other value: pi/2 where the
  lattice index sum is odd) or "random" (uniform in [0, 2 pi)). W runs differ
  in their seeds: run w draws from default_rng(seed + w), axes first, then
  the random phases.
* Spheres start at the spring's rest length, as everywhere else
  (place_dumbbells).

Everything here draws inputs only; the dynamics and the observables live
elsewhere.
"""
from __future__ import annotations

import math

import numpy as np

from .suspensions import Ensemble, Params, place_dumbbells

ELL_FIG1 = 5e-6          # m
OMEGA_FIG1 = 500.0       # 1/s
K0_FIG1 = 1e-3           # kg/s^2
MU_FIG1 = 1e-3           # kg/(m s)


def fig1_params(a_over_ell: float = 0.2, steps_per_period: int = 10_000) -> Params:
    """Model parameters printed for the aligned-pair experiment (Fig. 1),
    with dt = T / steps_per_period."""
    T = 2.0 * math.pi / OMEGA_FIG1
    return Params(a=a_over_ell * ELL_FIG1, eta=MU_FIG1, k=K0_FIG1, ell=ELL_FIG1, lam=0.1 * ELL_FIG1,
                  T=T, dt=T / steps_per_period)


def _unit(v: np.ndarray) -> np.ndarray:
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def lattice_indices(x: int) -> np.ndarray:
    """(x^3, 3) integer lattice indices in C order (last index fastest)."""
    g = np.arange(x)
    return np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)


def checkerboard_phases(idx: np.ndarray) -> np.ndarray:
    """0 where the index sum is even, pi/2 where it is odd: every nearest
    lattice neighbour has the other phase."""
    return (0.5 * math.pi) * (np.asarray(idx).sum(1) % 2).astype(np.float64)


def lattice_array(x: int, spacing: float, seed: int, phases: str = "checkerboard"):
    """One array: (R [S,3], N [S,3], phi [S]) with S = x^3 dumbbells."""
    if phases not in ("checkerboard", "random"):
        raise ValueError(f"phases must be 'checkerboard' or 'random', not {phases!r}")
    idx = lattice_indices(x)
    R = (idx - 0.5 * (x - 1)) * float(spacing)
    rng = np.random.default_rng(seed)
    N = _unit(rng.standard_normal(R.shape))
    phi = checkerboard_phases(idx) if phases == "checkerboard" else rng.uniform(0.0, 2.0 * math.pi, len(R))
    return R, N, phi


def array_runs(x: int, spacing: float, W: int, phases: str = "checkerboard", seed: int = 0,
               params: Params | None = None):
    """W arrays as one ensemble of W equal systems (system w drawn with seed
    + w), plus their stroke-averaged states. Returns (Ensemble, R [W,S,3],
    N [W,S,3], phi [W,S])."""
    params = params or fig1_params()
    Rs, Ns, phis, Xs = [], [], [], []
    for w in range(W):
        R, N, phi = lattice_array(x, spacing, seed + w, phases)
        Rs.append(R)
        Ns.append(N)
        phis.append(phi)
        Xs.append(place_dumbbells(R, N, phi, params))
    S = x ** 3
    ens = Ensemble(np.concatenate(Xs), np.concatenate(phis), np.full(W, S, dtype=np.int32), params,
                   np.full(W, x * float(spacing)), [seed + w for w in range(W)])
    return ens, np.stack(Rs), np.stack(Ns), np.stack(phis)


def rotation_pair(theta: float, q0: float, distance: float, phases=(0.0, 0.5 * math.pi)):
    """Two dumbbells in the x-y plane: sigma at the origin along x, rho at
    distance * (cos theta, sin theta, 0) with axis (q0, sqrt(1 - q0^2), 0).
    Returns (R [2,3], N [2,3], phi [2])."""
    if not -1.0 <= q0 <= 1.0:
        raise ValueError("q0 is a projection of unit vectors: |q0| <= 1")
    R = np.array([[0.0, 0.0, 0.0], [distance * math.cos(theta), distance * math.sin(theta), 0.0]])
    N = np.array([[1.0, 0.0, 0.0], [q0, math.sqrt(1.0 - q0 * q0), 0.0]])
    return R, N, np.asarray(phases, dtype=np.float64)


def rotation_pairs(thetas, q0: float, distance: float, params: Params | None = None):
    """One two-dumbbell system per angle, as an ensemble. Returns
    (Ensemble, R [n,2,3], N [n,2,3], phi [n,2])."""
    params = params or fig1_params()
    Rs, Ns, phis, Xs = [], [], [], []
    for th in thetas:
        R, N, phi = rotation_pair(float(th), q0, distance)
        Rs.append(R)
        Ns.append(N)
        phis.append(phi)
        Xs.append(place_dumbbells(R, N, phi, params))
    n = len(Rs)
    ens = Ensemble(np.concatenate(Xs), np.concatenate(phis), np.full(n, 2, dtype=np.int32), params,
                   np.full(n, 2.0 * distance), list(range(n)))
    return ens, np.stack(Rs), np.stack(Ns), np.stack(phis)
