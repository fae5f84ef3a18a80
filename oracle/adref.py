"""ctypes wrapper of the plain FP64 CPU oracle (adref.c).

TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's CPU
baseline leg may import this module. It shares no code with the GPU library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from pathlib import Path

import numpy as np

HERE = Path(__file__).resolve().parent
SRC = HERE / "adref.c"
LIB = HERE / "libadref.so"
# sin and cos stay separate libm calls, as written: without -fno-builtin-*
# gcc merges sin(x) and cos(x) into one sincos(x) call, whose last bit can
# differ from the separate calls
CFLAGS = ["-O2", "-fno-fast-math", "-ffp-contract=off", "-fno-builtin-sin", "-fno-builtin-cos",
          "-fno-builtin-sincos", "-fopenmp", "-std=c99", "-fPIC", "-shared"]


def build(force: bool = True) -> Path:
    """Compile adref.c with gcc (no fast-math, no FMA contraction)."""
    if force or not LIB.exists() or LIB.stat().st_mtime < SRC.stat().st_mtime:
        tmp = LIB.with_suffix(".so.tmp")
        subprocess.run(["gcc", *CFLAGS, str(SRC), "-o", str(tmp), "-lm"], check=True)
        os.replace(tmp, LIB)
    return LIB


class _Params(C.Structure):
    _fields_ = [("a", C.c_double), ("eta", C.c_double), ("k", C.c_double), ("ell", C.c_double),
                ("lam", C.c_double), ("T", C.c_double), ("dt", C.c_double),
                ("steric_k", C.c_double), ("steric_r", C.c_double),
                ("integrator", C.c_int32), ("tensor", C.c_int32),
                ("kT", C.c_double), ("seed", C.c_uint64)]


_lib = None
_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int64)


def lib():
    global _lib
    if _lib is None:
        if not LIB.exists():
            build()
        L = C.CDLL(str(LIB))
        P = C.POINTER(_Params)
        L.adref_forces.argtypes = [P, C.c_int64, _dp, _dp, C.c_double, _dp]
        L.adref_mobility.argtypes = [P, C.c_int64, _dp, _dp, _dp]
        L.adref_mobility_apply.argtypes = [P, C.c_int64, _dp, _dp, _dp]
        L.adref_step.argtypes = [P, C.c_int32, _ip, _dp, _dp, C.c_double, C.c_int64, C.c_int64]
        L.adref_mobility_rows.argtypes = [P, C.c_int64, _dp, _dp, C.c_int64, _ip, _dp]
        L.adref_mobility_dense.argtypes = [P, C.c_int64, _dp, _dp, _dp]
        L.adref_run.argtypes = [P, C.c_int32, _ip, _dp, _dp, C.c_double, C.c_int64, C.c_int64,
                                C.c_int64, _dp, _dp]
        L.adref_energy.argtypes = [P, C.c_int64, _dp, _dp, C.c_double]
        L.adref_energy.restype = C.c_double
        L.adref_rest_length.argtypes = [P, C.c_double, C.c_double]
        L.adref_rest_length.restype = C.c_double
        L.adref_sa_rhs.argtypes = [P, C.c_int64, _dp, _dp, _dp, _dp, _dp]
        L.adref_sa_run.argtypes = [P, C.c_int64, _dp, _dp, _dp, C.c_double, C.c_int64]
        L.adref_philox.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
        L.adref_gauss3.argtypes = [C.c_uint64, C.c_int64, C.c_int64, _dp]
        L.adref_set_threads.argtypes = [C.c_int]
        L.adref_max_threads.restype = C.c_int
        _lib = L
    return _lib


def _params(p, integrator: int = 0, tensor: int = 0, kT: float = 0.0, seed: int = 0) -> _Params:
    return _Params(p.a, p.eta, p.k, p.ell, p.lam, p.T, p.dt, p.steric_k, p.steric_r,
                   integrator, tensor, float(kT), int(seed))


def _d(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _arr(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what} returned {code}")
        self.code = code


def _check(code: int, what: str, allow_nonfinite: bool = False) -> int:
    if code != 0 and not (allow_nonfinite and code == -5):
        raise OracleError(code, what)
    return code


def set_threads(n: int) -> None:
    lib().adref_set_threads(int(n))


def max_threads() -> int:
    return int(lib().adref_max_threads())


def forces(p, X, phi, t: float, allow_nonfinite: bool = False) -> np.ndarray:
    X, phi = _arr(X), _arr(phi)
    F = np.empty_like(X)
    _check(lib().adref_forces(C.byref(_params(p)), X.shape[0], _d(X), _d(phi), float(t), _d(F)),
           "adref_forces", allow_nonfinite)
    return F


def mobility(p, X, F, tensor: int = 0, allow_nonfinite: bool = False) -> np.ndarray:
    X, F = _arr(X), _arr(F)
    u = np.empty_like(X)
    _check(lib().adref_mobility(C.byref(_params(p, tensor=tensor)), X.shape[0], _d(X), _d(F), _d(u)),
           "adref_mobility", allow_nonfinite)
    return u


def mobility_rows(p, X, F, rows, tensor: int = 0) -> np.ndarray:
    X, F = _arr(X), _arr(F)
    rows = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
    u = np.empty((rows.shape[0], 3), dtype=np.float64)
    _check(lib().adref_mobility_rows(C.byref(_params(p, tensor=tensor)), X.shape[0], _d(X), _d(F),
                                     rows.shape[0], rows.ctypes.data_as(_ip), _d(u)),
           "adref_mobility_rows")
    return u


def mobility_dense(p, X, F, tensor: int = 0) -> np.ndarray:
    X, F = _arr(X), _arr(F)
    u = np.empty_like(X)
    _check(lib().adref_mobility_dense(C.byref(_params(p, tensor=tensor)), X.shape[0], _d(X), _d(F),
                                      _d(u)), "adref_mobility_dense")
    return u


def energy(p, X, phi, t: float) -> float:
    X, phi = _arr(X), _arr(phi)
    return float(lib().adref_energy(C.byref(_params(p)), X.shape[0], _d(X), _d(phi), float(t)))


def rest_length(p, t: float, phi: float) -> float:
    return float(lib().adref_rest_length(C.byref(_params(p)), float(t), float(phi)))


def run(p, X, phi, nsteps: int, t0: float = 0.0, step0: int = 0, record_every: int = 0,
        S_per_sys=None, integrator: int = 0, tensor: int = 0, allow_nonfinite: bool = False,
        kT: float = 0.0, seed: int = 0):
    """Advance a copy of X by nsteps. Returns (X_new, centres[nrec,S,3], com[nrec,nsys,3], status)."""
    X = _arr(X).copy()
    phi = _arr(phi)
    N = X.shape[0]
    if S_per_sys is None:
        S_per_sys = np.array([N // 2], dtype=np.int64)
    S_per_sys = np.asarray(S_per_sys, dtype=np.int64)
    off = np.zeros(len(S_per_sys) + 1, dtype=np.int64)
    off[1:] = np.cumsum(2 * S_per_sys)
    nsys = len(S_per_sys)
    nrec = nsteps // record_every if record_every > 0 else 0
    cen = np.zeros((nrec, N // 2, 3)) if nrec else None
    com = np.zeros((nrec, nsys, 3)) if nrec else None
    code = lib().adref_run(C.byref(_params(p, integrator, tensor, kT, seed)), nsys, off.ctypes.data_as(_ip),
                           _d(X), _d(phi), float(t0), int(step0), int(nsteps), int(record_every),
                           _d(cen) if cen is not None else None, _d(com) if com is not None else None)
    _check(code, "adref_run", allow_nonfinite)
    return X, cen, com, code


def sa_rhs(p, R, N, phi):
    """Stroke-averaged far-field velocities (dR/dt, dN/dt) of dumbbells
    with centres R, unit axes N and phases phi (Sec. III, Eq. e:eom)."""
    R, N, phi = _arr(R), _arr(N), _arr(phi)
    dR, dN = np.empty_like(R), np.empty_like(N)
    _check(lib().adref_sa_rhs(C.byref(_params(p)), R.shape[0], _d(R), _d(N), _d(phi), _d(dR), _d(dN)),
           "adref_sa_rhs")
    return dR, dN


def sa_run(p, R, N, phi, dt, nsteps):
    """RK4 of the stroke-averaged equations; returns new (R, N)."""
    R, N, phi = _arr(R).copy(), _arr(N).copy(), _arr(phi)
    _check(lib().adref_sa_run(C.byref(_params(p)), R.shape[0], _d(R), _d(N), _d(phi), float(dt), int(nsteps)),
           "adref_sa_run")
    return R, N


def philox(ctr, key):
    """Philox4x32-10 block for a 4-word counter and a 2-word key."""
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().adref_philox(c, k, o)
    return [int(v) for v in o]


def gauss3(seed, i, n):
    z = np.empty(3)
    lib().adref_gauss3(int(seed), int(i), int(n), _d(z))
    return z
