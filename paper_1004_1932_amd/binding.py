"""Python binding of libad.so (include/ad.h): argument marshalling only.

Every step of the hot path runs in the HIP kernels of libad.so. PyTorch
supplies device memory (tensors) and streams; nothing here computes on the
CPU. If the library is missing or cannot be loaded, every call raises.
"""
from __future__ import annotations

import ctypes as C
from pathlib import Path

import numpy as np

LIB_PATH = Path(__file__).resolve().parent / "libad.so"

AD_OK, AD_EINVAL, AD_ENOMEM, AD_EDEVICE, AD_ESTATE, AD_ENONFINITE, AD_ERANGE = 0, -1, -2, -3, -4, -5, -6
AD_FP64, AD_FP64_TILED, AD_FP32C, AD_FP64_DENSE = 0, 1, 2, 3
AD_RK4, AD_HEUN = 0, 1
AD_OSEEN, AD_RPY = 0, 1
TENSORS = {"oseen": AD_OSEEN, "rpy": AD_RPY}

PRECISIONS = {"fp64": AD_FP64, "fp64_tiled": AD_FP64_TILED, "fp32c": AD_FP32C, "fp64_dense": AD_FP64_DENSE}
INTEGRATORS = {"rk4": AD_RK4, "heun": AD_HEUN}

# the exported entry points, in the order include/ad.h declares them
EXPORTS = ("ad_create", "ad_destroy", "ad_workspace_size", "ad_bind_workspace", "ad_set_launch",
           "ad_get_launch", "ad_set_state", "ad_get_state", "ad_forces", "ad_mobility_apply",
           "ad_step", "ad_run", "ad_check", "ad_use_graph", "ad_profile_pairs", "ad_profile_read",
           "ad_valu_probe", "ad_sa_rhs", "ad_sa_workspace_size", "ad_sa_run", "ad_mobility_apply_static",
           "ad_last_error")


class ad_params(C.Structure):
    _fields_ = [("a", C.c_double), ("eta", C.c_double), ("k", C.c_double), ("ell", C.c_double),
                ("lambda_", C.c_double), ("T", C.c_double), ("dt", C.c_double),
                ("steric_k", C.c_double), ("steric_r", C.c_double),
                ("precision", C.c_int32), ("integrator", C.c_int32), ("tensor", C.c_int32),
                ("reserved", C.c_int32), ("kT", C.c_double), ("seed", C.c_uint64)]


class ad_launch(C.Structure):
    _fields_ = [("ipl", C.c_int32), ("jchunk", C.c_int32), ("wg", C.c_int32), ("wj", C.c_int32),
                ("posmode", C.c_int32), ("fused", C.c_int32)]


AD_POS_HILO, AD_POS_SINGLE = 1, 2


class ADError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"[{code}] {message}")
        self.code = code


_lib = None


def lib():
    """Load libad.so; raises ImportError if it was not built."""
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(str(LIB_PATH))
        vp, i32, i64, dp = C.c_void_p, C.c_int32, C.c_int64, C.POINTER(C.c_double)
        L.ad_create.argtypes = [C.POINTER(ad_params), i32, C.POINTER(C.c_int32), C.POINTER(vp)]
        L.ad_destroy.argtypes = [vp]
        L.ad_workspace_size.argtypes = [vp, C.POINTER(C.c_uint64)]
        L.ad_bind_workspace.argtypes = [vp, vp, C.c_uint64]
        L.ad_set_launch.argtypes = [vp, C.POINTER(ad_launch)]
        L.ad_get_launch.argtypes = [vp, C.POINTER(ad_launch)]
        L.ad_set_state.argtypes = [vp, vp, vp, C.c_double, i64, vp]
        L.ad_get_state.argtypes = [vp, vp, dp, C.POINTER(C.c_int64), vp]
        L.ad_forces.argtypes = [vp, vp, C.c_double, vp, vp]
        L.ad_mobility_apply.argtypes = [vp, vp, vp, vp, vp]
        L.ad_step.argtypes = [vp, i64, vp]
        L.ad_run.argtypes = [vp, i64, i32, vp, vp, vp]
        L.ad_check.argtypes = [vp, vp]
        L.ad_use_graph.argtypes = [vp, i32]
        L.ad_profile_pairs.argtypes = [vp, i32]
        L.ad_profile_read.argtypes = [vp, dp, C.POINTER(C.c_int64)]
        L.ad_sa_rhs.argtypes = [C.POINTER(ad_params), i32, vp, vp, vp, vp, vp, vp]
        L.ad_sa_workspace_size.argtypes = [i32, C.POINTER(C.c_uint64)]
        L.ad_sa_run.argtypes = [C.POINTER(ad_params), i32, vp, vp, vp, C.c_double, i64, vp, C.c_uint64, vp]
        L.ad_valu_probe.argtypes = [i32, i32, i32, vp, vp, vp]
        L.ad_mobility_apply_static.argtypes = [C.POINTER(ad_params), i32, vp, vp, vp, vp]
        L.ad_last_error.argtypes = [vp]
        L.ad_last_error.restype = C.c_char_p
        for name in EXPORTS:
            if name != "ad_last_error":
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(code: int, ctx) -> int:
    if code != AD_OK:
        msg = lib().ad_last_error(ctx)
        raise ADError(code, msg.decode() if msg else "")
    return code


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _dev(t, name, shape=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous float64")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return C.c_void_p(t.data_ptr())


def make_params(p, precision="fp32c", integrator="rk4", tensor="oseen", kT=0.0, seed=0) -> ad_params:
    """ad_params from any object with a, eta, k, ell, lam, T, dt (steric_k,
    steric_r optional)."""
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    integ = INTEGRATORS[integrator] if isinstance(integrator, str) else int(integrator)
    ten = TENSORS[tensor] if isinstance(tensor, str) else int(tensor)
    lam = getattr(p, "lam", getattr(p, "lambda_", None))
    return ad_params(float(p.a), float(p.eta), float(p.k), float(p.ell), float(lam), float(p.T),
                     float(p.dt), float(getattr(p, "steric_k", 0.0)), float(getattr(p, "steric_r", 0.0)),
                     prec, integ, ten, 0, float(kT), int(seed))


# ---------------------------------------------------------------- 1:1 entry points

def ad_create(params: ad_params, S_per_sys) -> C.c_void_p:
    S = np.ascontiguousarray(np.asarray(S_per_sys, dtype=np.int32).reshape(-1))
    ctx = C.c_void_p()
    _check(lib().ad_create(C.byref(params), int(S.shape[0]), S.ctypes.data_as(C.POINTER(C.c_int32)),
                           C.byref(ctx)), None)
    return ctx


def ad_destroy(ctx) -> None:
    lib().ad_destroy(ctx)


def ad_workspace_size(ctx) -> int:
    n = C.c_uint64()
    _check(lib().ad_workspace_size(ctx, C.byref(n)), ctx)
    return int(n.value)


def ad_bind_workspace(ctx, ws) -> None:
    _check(lib().ad_bind_workspace(ctx, C.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size()), ctx)


def ad_set_launch(ctx, ipl=0, jchunk=0, wg=0, wj=0, posmode=0, fused=0) -> None:
    """Launch shape (ad_launch in include/ad.h). fused: 0 pair kernel and
    epilogue; 1 one stage kernel, every source in LDS; 2 the same with 64
    targets per work-group; 3 one stage kernel streaming the sources."""
    L = ad_launch(int(ipl), int(jchunk), int(wg), int(wj), int(posmode), int(fused))
    _check(lib().ad_set_launch(ctx, C.byref(L)), ctx)


def ad_get_launch(ctx) -> dict:
    L = ad_launch()
    _check(lib().ad_get_launch(ctx, C.byref(L)), ctx)
    return {"ipl": L.ipl, "jchunk": L.jchunk, "wg": L.wg, "wj": L.wj, "posmode": L.posmode, "fused": L.fused}


def ad_set_state(ctx, X, phi, t0=0.0, step0=0, stream=None) -> None:
    """X: device (N, 3) float64; phi: device (S,) float64."""
    _check(lib().ad_set_state(ctx, _dev(X, "X"), _dev(phi, "phi"), float(t0), int(step0), _stream(stream)), ctx)


def ad_get_state(ctx, X_out, stream=None):
    t0 = C.c_double()
    step = C.c_int64()
    _check(lib().ad_get_state(ctx, _dev(X_out, "X_out"), C.byref(t0), C.byref(step), _stream(stream)), ctx)
    return float(t0.value), int(step.value)


def ad_forces(ctx, X, t, F_out, stream=None) -> None:
    _check(lib().ad_forces(ctx, _dev(X, "X"), float(t), _dev(F_out, "F_out", X.shape), _stream(stream)), ctx)


def ad_mobility_apply(ctx, X, F, u_out, stream=None) -> None:
    _check(lib().ad_mobility_apply(ctx, _dev(X, "X"), _dev(F, "F", X.shape), _dev(u_out, "u_out", X.shape),
                                   _stream(stream)), ctx)


def ad_step(ctx, nsteps, stream=None) -> None:
    _check(lib().ad_step(ctx, int(nsteps), _stream(stream)), ctx)


def ad_run(ctx, nsteps, record_every, centres=None, com=None, stream=None) -> int:
    """Returns AD_OK, or AD_ENONFINITE / AD_ERANGE (not raised) when a flag was set."""
    cp = _dev(centres, "centres") if centres is not None else None
    mp = _dev(com, "com") if com is not None else None
    code = lib().ad_run(ctx, int(nsteps), int(record_every), cp, mp, _stream(stream))
    if code in (AD_ENONFINITE, AD_ERANGE):
        return code
    return _check(code, ctx)


def ad_check(ctx, stream=None) -> int:
    code = lib().ad_check(ctx, _stream(stream))
    if code in (AD_ENONFINITE, AD_ERANGE):
        return code
    return _check(code, ctx)


def ad_use_graph(ctx, enable: bool) -> None:
    _check(lib().ad_use_graph(ctx, 1 if enable else 0), ctx)


def ad_profile_pairs(ctx, enable: bool) -> None:
    _check(lib().ad_profile_pairs(ctx, 1 if enable else 0), ctx)


def ad_profile_read(ctx):
    """(summed pair-kernel milliseconds, launches) since ad_profile_pairs."""
    ms = C.c_double()
    n = C.c_int64()
    _check(lib().ad_profile_read(ctx, C.byref(ms), C.byref(n)), ctx)
    return float(ms.value), int(n.value)


def ad_valu_probe(kind: int, blocks: int, iters: int, sink, clk, stream=None) -> None:
    """Issue-rate probe (include/ad.h): sink float32 [blocks*256], clk int64 [2]
    zeroed, both device tensors."""
    import torch
    if sink.dtype != torch.float32 or sink.numel() < blocks * 256 or clk.dtype != torch.int64 or clk.numel() < 2:
        raise ValueError("sink: float32 [blocks*256], clk: int64 [2]")
    _check(lib().ad_valu_probe(int(kind), int(blocks), int(iters), C.c_void_p(sink.data_ptr()),
                               C.c_void_p(clk.data_ptr()), _stream(stream)), None)


def _sa_check(code: int, what: str) -> None:
    if code != AD_OK:
        raise ADError(code, what)


def ad_sa_rhs(params: ad_params, R, N, phi, dR_out, dN_out, stream=None) -> None:
    S = R.shape[0]
    _sa_check(lib().ad_sa_rhs(C.byref(params), int(S), _dev(R, "R", (S, 3)), _dev(N, "N", (S, 3)),
                              _dev(phi, "phi", (S,)), _dev(dR_out, "dR", (S, 3)), _dev(dN_out, "dN", (S, 3)),
                              _stream(stream)), "ad_sa_rhs")


def ad_sa_workspace_size(S: int) -> int:
    n = C.c_uint64()
    _sa_check(lib().ad_sa_workspace_size(int(S), C.byref(n)), "ad_sa_workspace_size")
    return int(n.value)


def ad_sa_run(params: ad_params, R, N, phi, dt, nsteps, workspace, stream=None) -> int:
    """Advance (R, N) in place; returns AD_OK or AD_ENONFINITE."""
    S = R.shape[0]
    code = lib().ad_sa_run(C.byref(params), int(S), _dev(R, "R", (S, 3)), _dev(N, "N", (S, 3)),
                           _dev(phi, "phi", (S,)), float(dt), int(nsteps), C.c_void_p(workspace.data_ptr()),
                           workspace.numel() * workspace.element_size(), _stream(stream))
    if code == AD_ENONFINITE:
        return code
    _sa_check(code, "ad_sa_run")
    return code


def ad_mobility_apply_static(params: ad_params, X, F, u_out, stream=None) -> None:
    """u = M(X) F for one system with no context, workspace or allocation
    (the library's own per-device scratch array)."""
    N = X.shape[0]
    code = lib().ad_mobility_apply_static(C.byref(params), int(N), _dev(X, "X", (N, 3)), _dev(F, "F", (N, 3)),
                                          _dev(u_out, "u_out", (N, 3)), _stream(stream))
    _check(code, None)


def ad_last_error(ctx=None) -> str:
    msg = lib().ad_last_error(ctx)
    return msg.decode() if msg else ""


# ---------------------------------------------------------------- owner of a context

class torch_device:
    """Make `device` current while a context binds its workspace."""

    def __init__(self, device):
        self.device = device

    def __enter__(self):
        import torch
        self._ctx = torch.cuda.device(self.device)
        return self._ctx.__enter__()

    def __exit__(self, *a):
        return self._ctx.__exit__(*a)


class Simulator:
    """A context plus its workspace tensor on one device."""

    def __init__(self, params, S_per_sys, precision="fp32c", integrator="rk4", device="cuda:0",
                 launch=None, graph=False, tensor="oseen", kT=0.0, seed=0):
        """launch: None (library default), a dict of ad_launch fields, or
        "tuned": for FP32C the autotuned shape of this size bucket (if any),
        for the plain FP64 forms the resident form up to 64 spheres per
        system, for the dense form the library default."""
        import torch
        self.device = torch.device(device)
        self.S_per_sys = np.asarray(S_per_sys, dtype=np.int32).reshape(-1)
        self.nsys = int(self.S_per_sys.shape[0])
        self.Stot = int(self.S_per_sys.sum())
        self.N = 2 * self.Stot
        self._p = make_params(params, precision, integrator, tensor, kT, seed)
        self._graph = bool(graph)
        if launch == "tuned":
            from .autotune import tuned_launch, tuned_launch_fp64
            if self._p.precision == AD_FP32C:
                launch = tuned_launch(self.S_per_sys)
            elif self._p.precision in (AD_FP64, AD_FP64_TILED):
                launch = tuned_launch_fp64(self.S_per_sys, steric=self._p.steric_k != 0.0)
            else:
                launch = None
        self.ctx = None
        self.ws = None
        self._create(launch)

    def _create(self, launch):
        if self.ctx is not None:
            ad_destroy(self.ctx)
        with torch_device(self.device):
            self.ctx = ad_create(self._p, self.S_per_sys)
            if launch:
                ad_set_launch(self.ctx, **launch)
            self._bind()
            if self._graph:
                ad_use_graph(self.ctx, True)

    def _bind(self):
        import torch
        nbytes = ad_workspace_size(self.ctx)
        self.ws = torch.empty((nbytes + 255) // 256 * 256 // 8, dtype=torch.float64, device=self.device)
        ad_bind_workspace(self.ctx, self.ws)

    def set_launch(self, **kw):
        """Change the launch shape. If the workspace is too small for it, the
        context is recreated with a larger one and the state must be set
        again."""
        try:
            ad_set_launch(self.ctx, **kw)
        except ADError as e:
            if e.code != AD_ENOMEM:
                raise
            self._create(kw)

    @property
    def launch(self):
        return ad_get_launch(self.ctx)

    def set_state(self, X, phi, t0=0.0, step0=0):
        import torch
        X = torch.as_tensor(X, dtype=torch.float64).to(self.device).contiguous()
        if isinstance(phi, torch.Tensor):
            phi = phi.to(self.device, torch.float64).contiguous()
        else:
            phi = torch.as_tensor(np.asarray(phi, dtype=np.float64)).to(self.device).contiguous()
        ad_set_state(self.ctx, X, phi, t0, step0)

    def get_state(self):
        import torch
        X = torch.empty((self.N, 3), dtype=torch.float64, device=self.device)
        t0, step = ad_get_state(self.ctx, X)
        return X, t0, step

    def forces(self, X, t):
        import torch
        X = torch.as_tensor(X, dtype=torch.float64).to(self.device).contiguous()
        F = torch.empty_like(X)
        ad_forces(self.ctx, X, t, F)
        return F

    def mobility(self, X, F):
        import torch
        X = torch.as_tensor(X, dtype=torch.float64).to(self.device).contiguous()
        F = torch.as_tensor(F, dtype=torch.float64).to(self.device).contiguous()
        u = torch.empty_like(X)
        ad_mobility_apply(self.ctx, X, F, u)
        return u

    def step(self, nsteps):
        ad_step(self.ctx, nsteps)

    def run(self, nsteps, record_every):
        import torch
        nrec = nsteps // record_every if record_every > 0 else 0
        cen = torch.empty((max(nrec, 1), self.Stot, 3), dtype=torch.float64, device=self.device)
        com = torch.empty((max(nrec, 1), self.nsys, 3), dtype=torch.float64, device=self.device)
        code = ad_run(self.ctx, nsteps, record_every, cen, com)
        return cen[:nrec], com[:nrec], code

    def check(self):
        return ad_check(self.ctx)

    def use_graph(self, enable=True):
        ad_use_graph(self.ctx, enable)

    def close(self):
        if self.ctx is not None:
            ad_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class StrokeAveraged:
    """Stroke-averaged far-field dynamics of S dumbbells on one device
    (Sec. III): device state R, N, phi plus the RK4 workspace."""

    def __init__(self, params, R, N, phi, device="cuda:0"):
        import torch
        self.device = torch.device(device)
        self._p = make_params(params)
        self.R = torch.as_tensor(R, dtype=torch.float64).to(self.device).contiguous()
        self.N = torch.as_tensor(N, dtype=torch.float64).to(self.device).contiguous()
        self.phi = torch.as_tensor(phi, dtype=torch.float64).to(self.device).contiguous()
        S = self.R.shape[0]
        nb = ad_sa_workspace_size(S)
        self.ws = torch.empty((nb + 255) // 256 * 32, dtype=torch.float64, device=self.device)

    def rhs(self):
        import torch
        dR, dN = torch.empty_like(self.R), torch.empty_like(self.N)
        ad_sa_rhs(self._p, self.R, self.N, self.phi, dR, dN)
        return dR, dN

    def run(self, dt, nsteps):
        return ad_sa_run(self._p, self.R, self.N, self.phi, dt, nsteps, self.ws)
