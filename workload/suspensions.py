"""Initial conditions for suspensions of active spring dumbbells.

Recipe (the paper's model, Sec. II; initial placement, Sec. V):
  * S dumbbells, N = 2S spheres of radius a; dumbbell s owns spheres 2s and
    2s+1 (0-based form of the paper's pair (2s-1, 2s)).
  * Dumbbell centres uniform in a free-space cube of side `side` centred at
    the origin; orientations uniform on the unit sphere (normalised standard
    normal 3-vector); stroke phases uniform in [0, 2*pi).
  * Spheres start at the spring's potential minimum, d(0) = L(0)
    = ell + lam*sin(phi), placed at R -/+ N*L(0)/2 (App. A, Eq. for the
    bead coordinates in terms of R and N).
  * Random sequential addition: a dumbbell is redrawn (centre and orientation,
    phase kept) while one of its spheres lies closer than 2a to a sphere that
    is already placed. The Oseen tensor is only meaningful for r > 2a
    (Sec. II), so overlapping draws are excluded. `exclusion=False` gives the
    literal uniform draw.
  * numpy default_rng(seed) (PCG64). Per dumbbell: draw phi, then draw
    (centre, orientation) until accepted.

Ensembles: system sizes S_b = default_rng(0).integers(16, 401, nsys); system b
is drawn with default_rng(1 + b) in a cube of side (2 S_b / density)^(1/3).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np


@dataclass(frozen=True)
class Params:
    """Model parameters (Sec. II) plus the integrator step and an optional
    steric repulsion that the paper does not have (force steric_k*(steric_r-r)
    along the separation for r < steric_r; steric_k = 0 disables it)."""
    a: float = 1.0          # sphere radius
    eta: float = 1.0        # viscosity
    k: float = 1.0          # spring constant k_0
    ell: float = 4.0        # mean dumbbell length
    lam: float = 1.0        # stroke amplitude lambda
    T: float = 100.0        # stroke period, omega = 2 pi / T
    dt: float = 0.01        # RK4 step
    steric_k: float = 0.0   # steric repulsion strength (0: off)
    steric_r: float = 2.0   # steric contact distance (2a)


@dataclass
class Suspension:
    X: np.ndarray           # (N, 3) float64 sphere positions
    phi: np.ndarray         # (S,) float64 stroke phases
    params: Params
    side: float
    seed: int
    min_pair_distance: float = float("nan")

    @property
    def S(self) -> int:
        return int(self.phi.shape[0])

    @property
    def N(self) -> int:
        return int(self.X.shape[0])


@dataclass
class Ensemble:
    X: np.ndarray               # (sum N_b, 3) float64, systems concatenated
    phi: np.ndarray             # (sum S_b,) float64
    S_per_sys: np.ndarray       # (nsys,) int32
    params: Params
    sides: np.ndarray           # (nsys,) float64
    seeds: list = field(default_factory=list)

    @property
    def nsys(self) -> int:
        return int(self.S_per_sys.shape[0])

    @property
    def sphere_offsets(self) -> np.ndarray:
        off = np.zeros(self.nsys + 1, dtype=np.int64)
        off[1:] = np.cumsum(2 * self.S_per_sys.astype(np.int64))
        return off

    def system(self, b: int) -> Suspension:
        off = self.sphere_offsets
        s0 = int(off[b] // 2)
        return Suspension(self.X[off[b]:off[b + 1]].copy(),
                          self.phi[s0:s0 + int(self.S_per_sys[b])].copy(),
                          self.params, float(self.sides[b]), self.seeds[b])


def place_dumbbells(centres: np.ndarray, orients: np.ndarray, phi: np.ndarray,
                    params: Params, t0: float = 0.0) -> np.ndarray:
    """Sphere positions for dumbbells at rest: R -/+ N*L(t0)/2 with
    L(t0) = ell + lam*sin(omega*t0 + phi). `orients` need not be normalised."""
    centres = np.asarray(centres, dtype=np.float64).reshape(-1, 3)
    orients = np.asarray(orients, dtype=np.float64).reshape(-1, 3)
    phi = np.asarray(phi, dtype=np.float64).reshape(-1)
    nrm = orients / np.linalg.norm(orients, axis=1, keepdims=True)
    omega = 2.0 * math.pi / params.T
    L0 = params.ell + params.lam * np.sin(omega * t0 + phi)
    X = np.empty((2 * centres.shape[0], 3), dtype=np.float64)
    X[0::2] = centres - 0.5 * L0[:, None] * nrm
    X[1::2] = centres + 0.5 * L0[:, None] * nrm
    return X


class _Grid:
    """Uniform hash grid for the random-sequential-addition overlap test."""

    def __init__(self, cell: float):
        self.cell = cell
        self.cells: dict = {}

    def _key(self, p):
        c = self.cell
        return (math.floor(p[0] / c), math.floor(p[1] / c), math.floor(p[2] / c))

    def too_close(self, p, rmin2: float) -> bool:
        kx, ky, kz = self._key(p)
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    lst = self.cells.get((kx + dx, ky + dy, kz + dz))
                    if not lst:
                        continue
                    for q in lst:
                        ddx = p[0] - q[0]
                        ddy = p[1] - q[1]
                        ddz = p[2] - q[2]
                        if ddx * ddx + ddy * ddy + ddz * ddz < rmin2:
                            return True
        return False

    def add(self, p):
        self.cells.setdefault(self._key(p), []).append((p[0], p[1], p[2]))


def _draw_system(S: int, side: float, seed: int, params: Params,
                 exclusion: bool, max_tries: int = 100000, rmin: float | None = None):
    rng = np.random.default_rng(seed)
    rmin = 2.0 * params.a if rmin is None else float(rmin)
    grid = _Grid(max(rmin, 1e-12))
    omega = 2.0 * math.pi / params.T
    X = np.empty((2 * S, 3), dtype=np.float64)
    phi = np.empty(S, dtype=np.float64)
    half = 0.5 * side
    for s in range(S):
        phi[s] = rng.uniform(0.0, 2.0 * math.pi)
        L0 = params.ell + params.lam * math.sin(omega * 0.0 + phi[s])
        for _ in range(max_tries):
            c = rng.uniform(-half, half, 3)
            n = rng.standard_normal(3)
            nn = math.sqrt(float(n @ n))
            if nn == 0.0:
                continue
            n = n / nn
            p0 = c - 0.5 * L0 * n
            p1 = c + 0.5 * L0 * n
            if exclusion and (grid.too_close(p0, rmin * rmin) or grid.too_close(p1, rmin * rmin)):
                continue
            break
        else:
            raise RuntimeError(f"could not place dumbbell {s} of {S} in side {side}")
        X[2 * s] = p0
        X[2 * s + 1] = p1
        if exclusion:
            grid.add(p0)
            grid.add(p1)
    return X, phi


def min_pair_distance(X: np.ndarray, block: int = 2048) -> float:
    """Smallest distance between two distinct spheres (brute force, blocked)."""
    N = X.shape[0]
    best = math.inf
    for i0 in range(0, N, block):
        xi = X[i0:i0 + block]
        d2 = ((xi[:, None, :] - X[None, :, :]) ** 2).sum(-1)
        idx = np.arange(i0, min(i0 + block, N))
        d2[np.arange(len(idx)), idx] = math.inf
        best = min(best, float(d2.min()))
    return math.sqrt(best)


def make_single(S: int, side: float, seed: int = 0, params: Params | None = None,
                exclusion: bool = True, with_min_distance: bool = False,
                rmin: float | None = None) -> Suspension:
    """One suspension; `rmin` overrides the exclusion distance 2a."""
    params = params or Params()
    X, phi = _draw_system(S, side, seed, params, exclusion, rmin=rmin)
    sus = Suspension(X, phi, params, float(side), seed)
    if with_min_distance:
        sus.min_pair_distance = min_pair_distance(X)
    return sus


def ensemble_sizes(nsys: int = 512, smin: int = 16, smax: int = 400, seed: int = 0) -> np.ndarray:
    return np.random.default_rng(seed).integers(smin, smax + 1, nsys).astype(np.int32)


def make_ensemble(nsys: int = 512, smin: int = 16, smax: int = 400, density: float = 0.02,
                  params: Params | None = None, exclusion: bool = True,
                  sizes: np.ndarray | None = None) -> Ensemble:
    params = params or Params()
    S_b = ensemble_sizes(nsys, smin, smax) if sizes is None else np.asarray(sizes, dtype=np.int32)
    Xs, phis, sides, seeds = [], [], [], []
    for b, S in enumerate(S_b):
        side = (2.0 * float(S) / density) ** (1.0 / 3.0)
        X, phi = _draw_system(int(S), side, 1 + b, params, exclusion)
        Xs.append(X)
        phis.append(phi)
        sides.append(side)
        seeds.append(1 + b)
    return Ensemble(np.concatenate(Xs), np.concatenate(phis), S_b, params,
                    np.asarray(sides), seeds)


# Named workloads. Parameters shared by all: a = eta = k = 1, ell = 4,
# lam = 1, T = 100, dt = 0.01; RK4.
PRESETS = {
    # name: (S, side, steps, steric)
    "n16": dict(S=8, side=40.0, steps=10_000),
    "n512": dict(S=256, side=120.0, steps=100_000),
    "n4096": dict(S=2048, side=240.0, steps=10_000),
    "n65536": dict(S=32768, side=800.0, steps=1_000, steric_k=100.0),
    "ens512": dict(nsys=512, smin=16, smax=400, density=0.02, steps=2_000),
}


def make_preset(name: str, seed: int = 0):
    spec = PRESETS[name]
    params = Params()
    if "steric_k" in spec:
        params = replace(params, steric_k=spec["steric_k"], steric_r=2.0 * params.a)
    if "nsys" in spec:
        return make_ensemble(spec["nsys"], spec["smin"], spec["smax"], spec["density"], params)
    return make_single(spec["S"], spec["side"], seed, params)
