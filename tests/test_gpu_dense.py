"""GPU parity of the dense baseline (AD_FP64_DENSE, the paper's assembled
full tensor, Sec. V) against the FP64 oracle.

The dense product sums each tensor row in column order (ascending source
sphere, x-y-z inside a sphere) in j-chunks, so it differs from the oracle's
pair-by-pair sum only in rounding order. Bar: relative velocity error
<= 1e-13 against both the oracle's matrix-free sum and its dense mode;
positions after 1000 RK4 or Heun steps of a dilute suspension within
1e-12 of the oracle's, relative to the displacement.
"""
import numpy as np
import pytest

import paper_1004_1932_amd as P
from workload import make_ensemble, make_preset, make_single

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def say(msg):
    print(msg, flush=True)


def relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("tensor", ["oseen", "rpy"])
@pytest.mark.parametrize("S,side,launch", [(1, 10.0, None), (8, 40.0, None), (150, 90.0, None),
                                           (150, 90.0, dict(jchunk=64)), (700, 150.0, None),
                                           (700, 150.0, dict(jchunk=1024))])
def test_dense_mobility_matches_oracle(oracle, S, side, launch, tensor):
    _torch()
    sus = make_single(S, side, 21)
    say(f"dense mobility S={S} {tensor} {launch}")
    F = np.random.default_rng(22).standard_normal(sus.X.shape)
    t = 1 if tensor == "rpy" else 0
    s = P.Simulator(sus.params, [sus.S], precision="fp64_dense", tensor=tensor, launch=launch)
    u = s.mobility(sus.X, F).cpu().numpy()
    assert relerr(u, oracle.mobility(sus.params, sus.X, F, tensor=t)) <= 1e-13
    assert relerr(u, oracle.mobility_dense(sus.params, sus.X, F, tensor=t)) <= 1e-13


def test_dense_ensemble_matches_oracle(oracle):
    """Uneven systems in one launch pair: each system's own tensor."""
    _torch()
    sizes = np.array([1, 16, 120, 3, 57, 64, 33, 90], dtype=np.int32)
    ens = make_ensemble(nsys=len(sizes), sizes=sizes)
    say("dense ensemble")
    F = np.random.default_rng(23).standard_normal(ens.X.shape)
    s = P.Simulator(ens.params, sizes, precision="fp64_dense")
    u = s.mobility(ens.X, F).cpu().numpy()
    off = ens.sphere_offsets
    for b in range(len(sizes)):
        sl = slice(off[b], off[b + 1])
        assert relerr(u[sl], oracle.mobility(ens.params, ens.X[sl], F[sl])) <= 1e-13, b


@pytest.mark.parametrize("integrator", ["rk4", "heun"])
def test_dense_trajectory_matches_oracle(oracle, integrator):
    _torch()
    sus = make_preset("n16")
    say(f"dense trajectory n16 {integrator}")
    s = P.Simulator(sus.params, [sus.S], precision="fp64_dense", integrator=integrator, graph=True)
    s.set_state(sus.X, sus.phi)
    cen, com, code = s.run(1000, 250)
    assert code == 0
    Xg = s.get_state()[0].cpu().numpy()
    Xo, ceno, como, _ = oracle.run(sus.params, sus.X, sus.phi, 1000, record_every=250,
                                   integrator=1 if integrator == "heun" else 0)
    assert relerr(Xg - sus.X, Xo - sus.X) <= 1e-12
    assert np.abs(com.cpu().numpy() - como).max() <= 1e-12 * max(1.0, np.abs(como).max())


def test_dense_step_equals_fp64_step_n512(oracle):
    """The N = 512 suspension, 20 RK4 steps: dense and AD_FP64 (bitwise the
    oracle) agree to rounding order."""
    _torch()
    sus = make_preset("n512")
    say("dense vs fp64 n512")
    out = {}
    for prec in ("fp64", "fp64_dense"):
        s = P.Simulator(sus.params, [sus.S], precision=prec, graph=True)
        s.set_state(sus.X, sus.phi)
        _, _, code = s.run(20, 10)
        assert code == 0
        out[prec] = s.get_state()[0].cpu().numpy()
    Xo, _, _, _ = oracle.run(sus.params, sus.X, sus.phi, 20)
    assert np.array_equal(out["fp64"], Xo)
    assert relerr(out["fp64_dense"] - sus.X, Xo - sus.X) <= 1e-12


def test_dense_coincident_spheres_raise_flag():
    _torch()
    sus = make_single(8, 30.0, 3)
    X = sus.X.copy()
    X[5] = X[2]
    s = P.Simulator(sus.params, [sus.S], precision="fp64_dense")
    s.set_state(X, sus.phi)
    _, _, code = s.run(2, 1)
    assert code == P.binding.AD_ENONFINITE
