"""The pair and array experiments of Sec. IV on the GPU: W runs (or the
angles of the rotation experiment) as one ensemble launch of the microscopic
model, the stroke-averaged equations on the GPU beside it.

Parity: the collective displacements are tiny (about 1e-6 ell per period at
spacing 10 ell, against positions of order 10 ell), the regime in which the
paper reports that a plain FP32 code failed (Sec. V). So the bar is on the
displacement over the measured period itself, not on the positions:
||dR_gpu - dR_oracle|| / ||dR_oracle|| over every dumbbell, dR = R(2T) - R(T),
with AD_FP64 bitwise and FP32C within 1e-3. The stroke-averaged GPU runs meet
the oracle's to 1e-10.

The last two tests repeat the oracle-level claims (test_oracle_arrays.py) at
the paper's array sizes (5x5x5 with W = 16; 3^3 to 9^3 with W = 10), on the
GPU only (the oracle would take many minutes there): values are not printed
in the paper, so they check the shapes of Figs. 3 and 4.
"""
import math

import numpy as np
import pytest

import paper_1004_1932_amd as P
from parity_metrics import check_fp32c
from paper_1004_1932_amd import observables as obs
from workload import array_runs, fig1_params, rotation_pairs

pytestmark = pytest.mark.gpu

SPP = 5000
# the fused stage kernel in its ensemble form (work list, 4-wave work-groups)
ENS_FUSED = {"fused": 1, "ipl": 1, "jchunk": 128, "posmode": 2, "wg": 64, "wj": 1}


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def say(msg):
    print(msg, flush=True)


def relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def gpu_micro(ens, periods, precision, launch):
    """Settling period, then `periods` periods; returns (X at T, X at the end)."""
    s = P.Simulator(ens.params, ens.S_per_sys, precision=precision, launch=launch, graph=True)
    s.set_state(ens.X, ens.phi)
    _, _, code = s.run(SPP, 0)
    assert code == 0
    X1 = s.get_state()[0].cpu().numpy()
    _, _, code = s.run(periods * SPP, 0)
    assert code == 0
    X2 = s.get_state()[0].cpu().numpy()
    s.close()
    return X1, X2


def gpu_sa(p, R1, N1, phi_runs, S_per_sys, periods):
    Rs, Ns, o = [], [], 0
    for b, Sb in enumerate(S_per_sys):
        sa = P.StrokeAveraged(p, R1[o:o + Sb], N1[o:o + Sb], phi_runs[b])
        assert sa.run(p.T / 20, 20 * periods) == 0
        Rs.append(sa.R.cpu().numpy())
        Ns.append(sa.N.cpu().numpy())
        o += Sb
    return np.concatenate(Rs), np.concatenate(Ns)


@pytest.mark.parametrize("precision,launch,tol", [("fp64", None, 0.0), ("fp32c", None, 1e-3),
                                                  ("fp32c", ENS_FUSED, 1e-3),
                                                  ("fp32c", dict(ENS_FUSED, posmode=1), 1e-3)])
def test_array_displacements_match_oracle(oracle, precision, launch, tol):
    """3x3x3 checkerboard arrays at spacing 10 ell, W = 4 runs in one launch."""
    _torch()
    p = fig1_params(0.2, SPP)
    ens, _, _, phi = array_runs(3, 10 * p.ell, 4, "checkerboard", seed=11, params=p)
    say(f"arrays {precision} {launch}")
    X1, X2 = gpu_micro(ens, 1, precision, launch)
    O1, _, _, _ = oracle.run(p, ens.X, ens.phi, SPP, S_per_sys=ens.S_per_sys)
    O2, _, _, _ = oracle.run(p, O1, ens.phi, SPP, t0=0.0, step0=SPP, S_per_sys=ens.S_per_sys)
    dg = obs.centres(X2) - obs.centres(X1)
    do = obs.centres(O2) - obs.centres(O1)
    err = relerr(dg, do)
    mg = obs.ensemble_msd(obs.centres(X2), obs.centres(X1), ens.S_per_sys)
    mo = obs.ensemble_msd(obs.centres(O2), obs.centres(O1), ens.S_per_sys)
    say(f"  displacement error {err:.2e}, msd {mg / p.ell ** 2:.6e} vs oracle {mo / p.ell ** 2:.6e} ell^2")
    if tol == 0.0:
        assert np.array_equal(X2, O2)
    else:
        assert err <= tol
        assert abs(mg / mo - 1) <= 2 * tol + tol * tol
    # the stroke-averaged equations from the settled state, GPU against oracle
    R1, N1 = obs.centres(X1), obs.axes(X1)
    Rs, Ns = gpu_sa(p, R1, N1, phi, ens.S_per_sys, 1)
    Ro, No, o = [], [], 0
    for b, Sb in enumerate(ens.S_per_sys):
        r, n = oracle.sa_run(p, R1[o:o + Sb], N1[o:o + Sb], phi[b], p.T / 20, 20)
        Ro.append(r)
        No.append(n)
        o += Sb
    assert relerr(Rs - R1, np.concatenate(Ro) - R1) <= 1e-10
    assert np.abs(Ns - np.concatenate(No)).max() <= 1e-12


@pytest.mark.parametrize("precision,launch,tol", [("fp64", None, 0.0), ("fp32c", None, 1e-3),
                                                  ("fp32c", ENS_FUSED, 1e-3)])
def test_rotation_pairs_match_oracle(oracle, precision, launch, tol):
    """Fig. 2 setup, one two-dumbbell system per angle in one launch:
    Delta q over five periods after settling, against the oracle's."""
    _torch()
    p = fig1_params(0.2, SPP)
    degs = (15, 75, 105, 165)
    ens, _, _, _ = rotation_pairs(np.radians(degs), 0.0, 5 * p.ell, params=p)
    say(f"rotation pairs {precision} {launch}")
    X1, X2 = gpu_micro(ens, 5, precision, launch)
    O1, _, _, _ = oracle.run(p, ens.X, ens.phi, SPP, S_per_sys=ens.S_per_sys)
    O2, _, _, _ = oracle.run(p, O1, ens.phi, 5 * SPP, t0=0.0, step0=SPP, S_per_sys=ens.S_per_sys)
    dq_g = obs.pair_projection(obs.axes(X2)) - obs.pair_projection(obs.axes(X1))
    dq_o = obs.pair_projection(obs.axes(O2)) - obs.pair_projection(obs.axes(O1))
    say(f"  dq gpu {dq_g}, oracle {dq_o}")
    if tol == 0.0:
        assert np.array_equal(X2, O2)
    else:
        assert np.abs(dq_g - dq_o).max() <= tol * np.abs(dq_o).max()


def array_msd(x, spacing_ell, W, phases, seed):
    """<<R(T)^2>> of W x^3 arrays (one launch), microscopic (FP32C, fused
    ensemble stage) and stroke-averaged (GPU), in units of ell^2."""
    p = fig1_params(0.2, SPP)
    ens, _, _, phi = array_runs(x, spacing_ell * p.ell, W, phases, seed=seed, params=p)
    X1, X2 = gpu_micro(ens, 1, "fp32c", ENS_FUSED)
    R1 = obs.centres(X1)
    Rs, _ = gpu_sa(p, R1, obs.axes(X1), phi, ens.S_per_sys, 1)
    m = obs.ensemble_msd(obs.centres(X2), R1, ens.S_per_sys) / p.ell ** 2
    s = obs.ensemble_msd(Rs, R1, ens.S_per_sys) / p.ell ** 2
    say(f"{x}^3 {phases} spacing {spacing_ell} ell, W = {W}: <<R(T)^2>> mic {m:.4e}, sa {s:.4e} ell^2, "
        f"sqrt ratio {math.sqrt(m / s):.3f}")
    return m, s


def test_array_msd_against_density():
    """Fig. 3: 5x5x5 arrays, W = 16, spacings 10 and 20 ell, both phase
    kinds. <<R(T)^2>> scales with nu = -4, checkerboard phases beat random
    ones, and the microscopic / stroke-averaged ratio is the same for every
    configuration."""
    _torch()
    out = {(ph, sp): array_msd(5, sp, 16, ph, 100) for ph in ("checkerboard", "random") for sp in (10, 20)}
    for phases in ("checkerboard", "random"):
        (m10, s10), (m20, s20) = out[phases, 10], out[phases, 20]
        assert abs(math.log2(s10 / s20) - 8) < 0.02
        assert abs(math.log2(m10 / m20) - 8) < 0.2
    for sp in (10, 20):
        for model in (0, 1):
            assert out["checkerboard", sp][model] > 1.3 * out["random", sp][model]
    shifts = [math.sqrt(m / s) for m, s in out.values()]
    assert max(shifts) / min(shifts) < 1.1 and 1.1 < min(shifts) < 1.6


def test_array_msd_against_number():
    """Fig. 4: x^3 arrays, x = 3, 5, 7, 9, spacing 10 ell, W = 10. The
    27-dumbbell array moves least, more dumbbells at the same density add
    little (9^3 within 30 % of 5^3), checkerboard phases beat random ones at
    every size, for both models."""
    _torch()
    out = {(ph, x): array_msd(x, 10, 10, ph, 200) for ph in ("checkerboard", "random") for x in (3, 5, 7, 9)}
    for ph in ("checkerboard", "random"):
        for model in (0, 1):
            v = [out[ph, x][model] for x in (3, 5, 7, 9)]
            assert v[0] == min(v), (ph, model, v)
            assert v[3] / v[1] < 1.3, (ph, model, v)
    for x in (3, 5, 7, 9):
        for model in (0, 1):
            assert out["checkerboard", x][model] > 1.3 * out["random", x][model]


def test_tuned_launch_on_lattice_ensembles(oracle):
    """The tuned launch of few-system lattice ensembles (their ":few" bucket
    or its size bucket) against the oracle: 3^3 and 7^3 lattices, W = 3,
    100 steps from rest, displacement within 1e-6."""
    _torch()
    from paper_1004_1932_amd.autotune import bucket_key, tuned_launch
    p = fig1_params(0.2, SPP)
    for x in (3, 7):
        ens, _, _, _ = array_runs(x, 10 * p.ell, 3, "checkerboard", seed=5, params=p)
        launch = tuned_launch(ens.S_per_sys)
        say(f"tuned {bucket_key(ens.S_per_sys)}: {launch}")
        assert launch is not None and launch.get("fused") in (1, 2, 4)
        s = P.Simulator(p, ens.S_per_sys, precision="fp32c", launch="tuned", graph=True)
        s.set_state(ens.X, ens.phi)
        _, _, code = s.run(100, 0)
        assert code == 0
        Xg = s.get_state()[0].cpu().numpy()
        s.close()
        Xo, _, _, _ = oracle.run(p, ens.X, ens.phi, 100, S_per_sys=ens.S_per_sys)
        check_fp32c(Xg - ens.X, Xo - ens.X, f"{x}^3 x 3: displacement")
