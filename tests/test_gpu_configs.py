"""The seeded workloads at their own sizes and lengths, on the launches the
benchmark uses, against stored FP64 oracle trajectories
(tests/golden/*_rk4.npz, written by tests/golden/make_config_goldens.py from
the oracle alone) or, for the 65536-sphere suspension, against oracle rows
and an oracle step computed here.

Bars: AD_FP64 bitwise; AD_FP32C relative centre-displacement drift <= 1e-4
at every record, relative velocity error <= 1e-6 per evaluation and the
per-sphere bound of parity_metrics.SPHERE_BAR.
"""
from __future__ import annotations

import json
from pathlib import Path

import numpy as np
import pytest

import paper_1004_1932_amd as P
from parity_metrics import DRIFT_BAR, check_fp32c, near_term_scale, relerr, sphere_err
from workload import Params, make_preset, make_single

pytestmark = pytest.mark.gpu

GOLDEN = Path(__file__).resolve().parent / "golden"


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def say(msg):
    print(msg, flush=True)


def golden(name):
    import hashlib
    path = GOLDEN / f"{name}_rk4.npz"
    man = json.loads((GOLDEN / "config_goldens.json").read_text())
    assert hashlib.sha256(path.read_bytes()).hexdigest() == man["files"][path.name]["sha256"], path
    with np.load(path, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def centres(X):
    return 0.5 * (X[0::2] + X[1::2])


def drifts(cen_gpu, cen_orc, R0):
    return [relerr(cen_gpu[r] - R0, cen_orc[r] - R0) for r in range(len(cen_orc))]


# ---------------------------------------------------------------- 512 spheres, 1e5 steps

def test_n512_fp64_bitwise_full_length():
    """S = 256, 1e5 RK4 steps in plain FP64: centres and centre of mass at
    every 1e4 steps and the final state bitwise equal to the oracle's."""
    _torch()
    g = golden("n512")
    sus = make_preset("n512")
    steps, rec = int(g["steps"]), int(g["record_every"])
    say(f"n512 fp64 {steps} steps")
    s = P.Simulator(sus.params, [sus.S], precision="fp64", graph=True)
    s.set_state(sus.X, sus.phi)
    cen, com, code = s.run(steps, rec)
    assert code == 0
    assert np.array_equal(s.get_state()[0].cpu().numpy(), g["X"])
    assert np.array_equal(cen.cpu().numpy(), g["centres"])
    assert np.array_equal(com.cpu().numpy(), g["com"])


def test_n512_fp32c_drift_full_length(oracle):
    """S = 256, 1e5 RK4 steps in the tuned FP32C launch: centre drift at every
    1e4 steps, and the velocity at the final state."""
    _torch()
    g = golden("n512")
    sus = make_preset("n512")
    steps, rec = int(g["steps"]), int(g["record_every"])
    s = P.Simulator(sus.params, [sus.S], precision="fp32c", launch="tuned", graph=True)
    say(f"n512 fp32c {steps} steps, launch {s.launch}")
    s.set_state(sus.X, sus.phi)
    cen, _, code = s.run(steps, rec)
    assert code == 0
    d = drifts(cen.cpu().numpy(), g["centres"], centres(sus.X))
    say(f"  drift per record {['%.2e' % x for x in d]}")
    assert max(d) <= DRIFT_BAR
    Xg = s.get_state()[0].cpu().numpy()
    F = oracle.forces(sus.params, Xg, sus.phi, steps * sus.params.dt)
    check_fp32c(s.mobility(Xg, F).cpu().numpy(), oracle.mobility(sus.params, Xg, F), "final-state velocity")


# ---------------------------------------------------------------- 4096 spheres, 1e4 steps

def test_n4096_fp32c_drift_full_length(oracle):
    """S = 2048, 1e4 RK4 steps in the launch the benchmark times (tuned):
    centre drift at every 1000 steps, and the velocity at the final state."""
    _torch()
    g = golden("n4096")
    sus = make_preset("n4096")
    steps, rec = int(g["steps"]), int(g["record_every"])
    s = P.Simulator(sus.params, [sus.S], precision="fp32c", launch="tuned", graph=True)
    say(f"n4096 fp32c {steps} steps, launch {s.launch}")
    s.set_state(sus.X, sus.phi)
    cen, com, code = s.run(steps, rec)
    assert code == 0
    cg = cen.cpu().numpy()
    R0 = centres(sus.X)
    d = drifts(cg, g["centres"], R0)
    say(f"  drift per record {['%.2e' % x for x in d]}")
    assert max(d) <= DRIFT_BAR
    # the drift of the worst dumbbell, on the scale of a typical displacement
    w = sphere_err(cg[-1] - R0, g["centres"][-1] - R0)
    say(f"  final per-dumbbell drift {w:.2e}")
    assert w <= DRIFT_BAR
    Xg = s.get_state()[0].cpu().numpy()
    F = oracle.forces(sus.params, Xg, sus.phi, steps * sus.params.dt)
    check_fp32c(s.mobility(Xg, F).cpu().numpy(), oracle.mobility(sus.params, Xg, F), "final-state velocity")


# ---------------------------------------------------------------- 512-system ensemble, 2000 steps

def test_ens512_tuned_full_length(oracle):
    """All 512 systems in the tuned launch for 2000 steps; 32 of them
    (largest, smallest, 30 random) against their oracle trajectories: drift
    per system at every 500 steps, and per-system velocity at the final
    state."""
    _torch()
    g = golden("ens512")
    ens = make_preset("ens512")
    steps, rec = int(g["steps"]), int(g["record_every"])
    s = P.Simulator(ens.params, ens.S_per_sys, precision="fp32c", launch="tuned", graph=True)
    say(f"ens512 fp32c {steps} steps, launch {s.launch}")
    s.set_state(ens.X, ens.phi)
    cen, _, code = s.run(steps, rec)
    assert code == 0
    cg = cen.cpu().numpy()
    Xg = s.get_state()[0].cpu().numpy()
    soff = np.concatenate([[0], np.cumsum(ens.S_per_sys.astype(np.int64))])
    off = ens.sphere_offsets
    t = steps * ens.params.dt
    F = np.concatenate([oracle.forces(ens.params, Xg[off[b]:off[b + 1]], ens.phi[soff[b]:soff[b + 1]], t)
                        for b in range(ens.nsys)])
    u = s.mobility(Xg, F).cpu().numpy()
    worst_d = worst_u = worst_s = 0.0
    go = 0
    for b, Sb in zip(g["systems"], g["S"]):
        b, Sb = int(b), int(Sb)
        assert Sb == int(ens.S_per_sys[b])
        ds = slice(int(soff[b]), int(soff[b + 1]))
        R0 = centres(ens.X[off[b]:off[b + 1]])
        d = max(drifts(cg[:, ds], g["centres"][:, go:go + Sb], R0))
        go += Sb
        sl = slice(int(off[b]), int(off[b + 1]))
        uo = oracle.mobility(ens.params, Xg[sl], F[sl])
        e, se = relerr(u[sl], uo), sphere_err(u[sl], uo)
        worst_d, worst_u, worst_s = max(worst_d, d), max(worst_u, e), max(worst_s, se)
        assert d <= DRIFT_BAR, (b, d)
        check_fp32c(u[sl], uo, f"system {b} (S={Sb}) drift {d:.2e}")
    say(f"  worst sampled system: drift {worst_d:.2e}, velocity {worst_u:.2e}, per-sphere {worst_s:.2e}")


# ---------------------------------------------------------------- 65536 spheres with contacts

def contact_suspension():
    """The 65536-sphere suspension drawn with exclusion distance 1.6 instead
    of 2a, so that several dozen pairs start inside the steric range (r < 2a)
    while the Oseen tensor stays regular."""
    p = Params(steric_k=100.0, steric_r=2.0)
    return make_single(32768, 800.0, 0, p, rmin=1.6)


def contacts(X, rc=2.0):
    from scipy.spatial import cKDTree
    return np.array(sorted(cKDTree(X).query_pairs(rc)), dtype=np.int64).reshape(-1, 2)


def test_n65536_steric_contacts(oracle):
    """Steric repulsion at full size with real contacts, tuned FP32C launch
    (candidate lists): at steps 2 and 40 the forces equal the oracle's
    bitwise and the velocities of 64 spheres (32 in contact, 32 random)
    match the oracle's rows; one step from the GPU's state at step 40
    matches a full oracle step, every sphere's displacement."""
    torch = _torch()
    sus = contact_suspension()
    p = sus.params
    pairs = contacts(sus.X)
    say(f"n65536 contacts at start: {len(pairs)} pairs, min r {np.linalg.norm(sus.X[pairs[:, 0]] - sus.X[pairs[:, 1]], axis=1).min():.3f}")
    assert len(pairs) >= 20
    s = P.Simulator(p, [sus.S], precision="fp32c", launch="tuned", graph=True)
    say(f"  launch {s.launch}")
    s.set_state(sus.X, sus.phi)
    done = 0
    for at in (2, 40):
        _, _, code = s.run(at - done, 0)
        assert code == 0
        done = at
        X = s.get_state()[0].cpu().numpy()
        t = at * p.dt
        now = contacts(X)
        rng = np.random.default_rng(7 + at)
        touch = np.unique(now.reshape(-1))
        rows = np.unique(np.concatenate([rng.choice(touch, min(32, len(touch)), replace=False),
                                         rng.choice(sus.N, 32, replace=False)]))
        F = s.forces(X, t).cpu().numpy()
        Fo = oracle.forces(p, X, sus.phi, t)
        assert np.array_equal(F, Fo)
        assert np.abs(Fo[touch]).max() > 1.0  # the steric force is acting
        u = s.mobility(X, Fo).cpu().numpy()
        uo = oracle.mobility_rows(p, X, Fo, rows)
        check_fp32c(u[rows], uo, f"step {at}: {len(now)} contacts, sampled rows")
    # one more GPU step (steric forces from the candidate lists) against a
    # full FP64 oracle step from the same state
    X40 = X
    _, _, code = s.run(1, 0)
    assert code == 0
    X41 = s.get_state()[0].cpu().numpy()
    Xo, _, _, _ = oracle.run(p, X40, sus.phi, 1, step0=40)
    # each sphere on the scale of its own displacement, the median one, and
    # what its near neighbours' terms would move it by in absolute value (the
    # terms of a contact pair's equal and opposite forces cancel, their FP32
    # rounding does not)
    near = p.dt * near_term_scale(X40, oracle.forces(p, X40, sus.phi, 40 * p.dt), p.eta)
    check_fp32c(X41 - X40, Xo - X40, "step 40 -> 41 displacement", extra=near)
    touch = np.unique(contacts(X40).reshape(-1))
    e = relerr((X41 - X40)[touch], (Xo - X40)[touch])
    say(f"  displacement of the {len(touch)} contacting spheres: rel err {e:.2e}")
    assert e <= 1e-6
    del s
    torch.cuda.empty_cache()
